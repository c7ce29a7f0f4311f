/*
 * microenv.h -- C ABI of the microenvironment solver in libmech.so (gfx950).
 *
 * The paper finds three load-imbalanced parallel regions in a PhysiCell iteration: the
 * microenvironment solver, the computation of the substrate gradients, and the cells'
 * velocity update (Section 5.2).  The first two are loops over the lines of a
 * 75 x 75 x 75 voxel mesh (Section 5.2, the listing of the solver's parallel loop);
 * mech.h holds the third.  The paper prints no equation for the solver.  What this
 * library computes is its reading of PhysiCell's solver:
 *
 *   Each substrate s has a density rho_s on nx x ny x nz cubic voxels of edge dx,
 *   stored x fastest: rho[s][(k ny + j) nx + i].  It obeys the diffusion-decay equation
 *   d rho / dt = D_s lap(rho) - lambda_s rho, with no flux through the outer faces.  One
 *   time step dt is three implicit (backward Euler) one-dimensional solves, along x,
 *   then y, then z, each carrying a third of the decay: along an axis of n voxels, with
 *   r = D_s dt / dx^2 and b = 1 + lambda_s dt / 3, the new values u of every mesh line
 *   solve  -r u_{i-1} + (b + 2r) u_i - r u_{i+1} = rho_i  inside, with the diagonal
 *   b + r on the two face rows (no flux through the wall) and b u = rho when n = 1.
 *
 *   The gradient of every substrate along every axis is the central difference
 *   (rho_{i+1} - rho_{i-1}) / (2 dx) inside, the one-sided difference on the first and
 *   last voxel of a line, and 0 along an axis of one voxel: grad[s][axis][voxel].
 *
 * Conventions are those of mech.h: MECH_OK or a negative MECH_E_* code, the text of the
 * last error from mech_last_error(), host arrays copied, device memory owned by the
 * handle until destroy_microenvironment, asynchronous calls on the handle's stream whose
 * device faults surface as MECH_E_DEVICE at the next synchronising call, one host thread
 * per handle at a time.  Units: um, min.
 */
#ifndef MECH_MICROENV_H
#define MECH_MICROENV_H

#include <stdint.h>

#include "mech.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MECH_MAX_SUBSTRATES 16

typedef struct MechMicroenvParams {
    int32_t abi_version;        /* MECH_ABI_VERSION                                     */
    int32_t n_substrates;       /* 1..MECH_MAX_SUBSTRATES                               */
    int32_t dims[3];            /* voxels per axis, each 1..4096; product < 2^31        */
    int32_t reserved;           /* must be 0                                             */
    double voxel_size;          /* dx, um (> 0)                                          */
    double dt;                  /* min (>= 0)                                            */
    double diffusion[MECH_MAX_SUBSTRATES];  /* D_s >= 0, um^2/min (first n_substrates)  */
    double decay[MECH_MAX_SUBSTRATES];      /* lambda_s >= 0, 1/min                      */
} MechMicroenvParams;

typedef struct MechMicroenv MechMicroenv;

/* Create a mesh on the current HIP device.
 *   density     n_substrates x nx*ny*nz doubles, [s][z][y][x], or NULL for zeros
 *   hip_stream  hipStream_t to run on, or NULL for a stream the handle owns
 * MECH_E_INVALID for bad parameters or a non-finite density; MECH_E_NOMEM if the device
 * memory (8 bytes x 4 values per voxel and substrate) cannot be had.  On error *out is
 * NULL and nothing is left allocated. */
int create_microenvironment(const MechMicroenvParams* params, const double* density, void* hip_stream,
                            MechMicroenv** out);

/* Enqueue n_steps solver steps (x, y and z solves each) and return.  After the first
 * call each step is one launch of a captured HIP graph.  Makes no allocation. */
int microenvironment_step(MechMicroenv* env, int64_t n_steps);

/* Enqueue the gradient computation from the current densities (asynchronous). */
int microenvironment_gradients(MechMicroenv* env);

/* Wait for the stream and copy the densities ([s][z][y][x], n_values = n_substrates x
 * voxels) or the gradients ([s][axis][z][y][x], n_values = 3 x n_substrates x voxels)
 * to the host.  MECH_E_INVALID if n_values does not match; MECH_E_NONFINITE if a value
 * read back is NaN or Inf. */
int read_density(MechMicroenv* env, double* density, int64_t n_values);
int read_gradients(MechMicroenv* env, double* grad, int64_t n_values);

/* Replace the densities (host array as in create_microenvironment; waits for the
 * stream first). */
int write_density(MechMicroenv* env, const double* density, int64_t n_values);

/* Run n_steps steps followed by one gradient computation with direct launches and HIP
 * events on the handle's stream around each kernel; on return ms[0..2] hold the mean
 * ms per launch of the x, y and z solves and ms[3] of the gradient kernel.  Same results
 * as microenvironment_step + microenvironment_gradients.  Synchronises. */
int microenvironment_profile(MechMicroenv* env, int64_t n_steps, double ms[4]);

/* Device addresses of the densities and gradients (layouts above), valid until
 * destroy_microenvironment; for callers that read them on the device. */
int microenvironment_device_arrays(MechMicroenv* env, double** density, double** grad);

/* hipStream_t the handle runs on. */
void* microenvironment_stream(MechMicroenv* env);

/* Wait for the stream and free everything the handle owns.  NULL is a no-op. */
int destroy_microenvironment(MechMicroenv* env);

#ifdef __cplusplus
}
#endif

#endif /* MECH_MICROENV_H */
