/*
 * diffusion_oracle.c -- plain, slow CPU oracle for the microenvironment solver and the
 * gradient computation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg load this library; the product path (the HIP library) never does and
 * shares no code with it.
 *
 * The paper names the two regions -- the microenvironment solver and the computation of
 * the substrate gradients -- as the first two of the three load-imbalanced parallel
 * regions of a PhysiCell iteration, and shows that both are loops over the z and then
 * y lines of a 75 x 75 x 75 voxel mesh (Section 5.2, the listing of the solver's
 * parallel loop).  It prints no equation for either.  What is computed here is the
 * solver as this project reads it (the BioFVM method PhysiCell calls):
 *
 *   Each substrate s has a density rho_s on a uniform mesh of nx x ny x nz cubic voxels
 *   of edge dx, stored x fastest: rho[s][(k * ny + j) * nx + i].  It obeys the
 *   diffusion-decay equation  d rho / dt = D_s lap(rho) - lambda_s rho  with no flux
 *   through the outer faces.  One time step dt is the locally one-dimensional (LOD)
 *   splitting: three implicit (backward Euler) one-dimensional solves, along x, then y,
 *   then z, each carrying a third of the decay.  Along an axis with n voxels, with
 *   r = D_s dt / dx^2 and b = 1 + lambda_s dt / 3, the new values u of a line solve
 *
 *     (b + r) u_0 - r u_1                       = rho_0            (first voxel)
 *     -r u_{i-1} + (b + 2r) u_i - r u_{i+1}     = rho_i            (0 < i < n-1)
 *     -r u_{n-2} + (b + r) u_{n-1}              = rho_{n-1}        (last voxel)
 *
 *   (the face rows are the interior row with the missing neighbour's flux removed: no
 *   flux through the wall), and b u_0 = rho_0 when n = 1.  Each system is solved by the
 *   Thomas algorithm (forward elimination, back substitution), written out below.
 *
 *   Gradient: for every voxel, substrate and axis, the central difference
 *   (rho_{i+1} - rho_{i-1}) / (2 dx) inside, the one-sided difference
 *   (rho_1 - rho_0) / dx on the first and (rho_{n-1} - rho_{n-2}) / dx on the last voxel
 *   of a line, and 0 along an axis with one voxel.  Stored grad[s][axis][voxel].
 *
 * Compiled with -ffp-contract=off: every result is the IEEE value of the expression as
 * written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define DIFF_MAX_SUBSTRATES 16

typedef struct {
    int32_t dims[3];            /* nx, ny, nz */
    int32_t n_substrates;
    double dx;                  /* voxel edge, um */
    double dt;                  /* time step, min */
    double diffusion[DIFF_MAX_SUBSTRATES];  /* D_s, um^2/min */
    double decay[DIFF_MAX_SUBSTRATES];      /* lambda_s, 1/min */
} DiffOracleParams;

/* Solve one line of n values, spaced `stride` apart from `u`, in place: the system above
 * with off-diagonal -r and diagonal b + 2r (b + r on the face rows).  cp holds the
 * eliminated upper diagonal of the line (n entries of scratch). */
static void thomas_line(double* u, int64_t stride, int n, double r, double b, double* cp)
{
    if (n == 1) {
        u[0] = u[0] / b;
        return;
    }
    /* forward elimination: row i becomes u_i + cp_i u_{i+1} = y_i */
    double diag = b + r;
    cp[0] = -r / diag;
    u[0] = u[0] / diag;
    for (int i = 1; i < n; ++i) {
        diag = (i == n - 1) ? b + r : b + 2.0 * r;
        double denom = diag - (-r) * cp[i - 1];
        cp[i] = (i == n - 1) ? 0.0 : -r / denom;
        u[i * stride] = (u[i * stride] - (-r) * u[(i - 1) * stride]) / denom;
    }
    /* back substitution */
    for (int i = n - 2; i >= 0; --i)
        u[i * stride] = u[i * stride] - cp[i] * u[(i + 1) * stride];
}

/* One LOD sweep along `axis` (0 x, 1 y, 2 z) of every line of every substrate. */
static void sweep(const DiffOracleParams* p, double* rho, int axis)
{
    const int nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
    const int64_t V = (int64_t)nx * ny * nz;
    const int n = p->dims[axis];
    const int64_t stride = axis == 0 ? 1 : axis == 1 ? nx : (int64_t)nx * ny;
    /* the lines: every voxel whose coordinate along `axis` is 0 starts one */
    const int na = axis == 0 ? ny : nx;     /* the two other axes, faster first */
    const int nb = axis == 2 ? ny : nz;
    for (int s = 0; s < p->n_substrates; ++s) {
        const double r = p->diffusion[s] * p->dt / (p->dx * p->dx);
        const double b = 1.0 + p->decay[s] * p->dt / 3.0;
        double* base = rho + (int64_t)s * V;
#pragma omp parallel
        {
            double* cp = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for collapse(2) schedule(static)
            for (int lb = 0; lb < nb; ++lb) {
                for (int la = 0; la < na; ++la) {
                    int64_t start;
                    if (axis == 0) start = ((int64_t)lb * ny + la) * nx;         /* (j, k) */
                    else if (axis == 1) start = (int64_t)lb * nx * ny + la;       /* (i, k) */
                    else start = (int64_t)lb * nx + la;                           /* (i, j) */
                    thomas_line(base + start, stride, n, r, b, cp);
                }
            }
            free(cp);
        }
    }
}

static int check(const DiffOracleParams* p)
{
    if (p->n_substrates < 1 || p->n_substrates > DIFF_MAX_SUBSTRATES) return -1;
    for (int a = 0; a < 3; ++a)
        if (p->dims[a] < 1) return -1;
    if (!(p->dx > 0.0) || !(p->dt >= 0.0)) return -1;
    for (int s = 0; s < p->n_substrates; ++s)
        if (!(p->diffusion[s] >= 0.0) || !(p->decay[s] >= 0.0)) return -1;
    return 0;
}

/* n_steps LOD steps of the diffusion-decay equation, in place on rho[s][z][y][x]. */
int32_t oracle_diffusion_step(const DiffOracleParams* p, double* rho, int64_t n_steps)
{
    if (check(p) != 0 || n_steps < 0) return -1;
    for (int64_t t = 0; t < n_steps; ++t) {
        sweep(p, rho, 0);
        sweep(p, rho, 1);
        sweep(p, rho, 2);
    }
    return 0;
}

/* One sweep alone (for the tests of the one-dimensional solves). */
int32_t oracle_diffusion_sweep(const DiffOracleParams* p, double* rho, int32_t axis)
{
    if (check(p) != 0 || axis < 0 || axis > 2) return -1;
    sweep(p, rho, axis);
    return 0;
}

/* Gradient of every substrate along every axis: grad[s][axis][voxel]. */
int32_t oracle_gradients(const DiffOracleParams* p, const double* rho, double* grad)
{
    if (check(p) != 0) return -1;
    const int nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
    const int64_t V = (int64_t)nx * ny * nz;
    const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
    for (int s = 0; s < p->n_substrates; ++s) {
        const double* u = rho + (int64_t)s * V;
        for (int axis = 0; axis < 3; ++axis) {
            double* g = grad + ((int64_t)s * 3 + axis) * V;
            const int n = p->dims[axis];
            const int64_t st = stride[axis];
#pragma omp parallel for collapse(2) schedule(static)
            for (int k = 0; k < nz; ++k) {
                for (int j = 0; j < ny; ++j) {
                    for (int i = 0; i < nx; ++i) {
                        const int64_t v = ((int64_t)k * ny + j) * nx + i;
                        const int c = axis == 0 ? i : axis == 1 ? j : k;
                        double val;
                        if (n == 1) val = 0.0;
                        else if (c == 0) val = (u[v + st] - u[v]) / p->dx;
                        else if (c == n - 1) val = (u[v] - u[v - st]) / p->dx;
                        else val = (u[v + st] - u[v - st]) / (2.0 * p->dx);
                        g[v] = val;
                    }
                }
            }
        }
    }
    return 0;
}
