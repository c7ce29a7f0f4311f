/*
 * mech.h -- C ABI of the MI355X (gfx950) agent-mechanics library, libmech.so.
 *
 * The library advances a population of spherical cells with the mechanics step of a
 * PhysiCell-style agent-based simulation: the region the paper calls "update
 * velocity", which it finds to dominate and to degrade as cells lose spatial locality
 * (Sections 4.1 and 5.4).  One step:
 *   a1  voxel of every cell on a uniform grid of edge h (anchored at domain_lo, x fastest)
 *   a2  voxel histogram
 *   a3  exclusive scan of the counts and the list of occupied voxels (the paper's
 *       non-empty voxel list, Section 5.4)
 *   a4  order of the cells inside each voxel: by x slab (each voxel cut into 4 slabs
 *       along x), then by ascending cell id (bit-exact order)
 *   a5  gather of the cell state into that voxel order, so that cells close in space
 *       are close in memory (the layout the paper recommends, Sections 5.4 and 6)
 *   a6  velocity of each cell: sum over the cells of the 27 surrounding voxels of
 *         w = c_rep (1 - d/R)^2 [d < R] - C[t_i][t_j] (1 - d/R_A)^2,  along (x_i - x_j)/d,
 *       with R = r_i + r_j, R_A = rel_adh_distance * R, for pairs with 0 < d^2 < R_A^2
 *   a7  two-step Adams-Bashforth update x += dt (1.5 v - 0.5 v_prev), reflecting walls
 *       (mirror at each face, then clamp), v_prev <- v
 * The force law, the overdamped velocity, the Adams-Bashforth update and the walls are
 * not printed in the paper; they are the method as this library defines it.
 *
 * Conventions
 *   - Every int-returning call returns MECH_OK (0) or a negative MECH_E_* code; the
 *     text of the last error on the calling thread is mech_last_error().
 *   - Host arrays passed in are copied; the caller keeps ownership.  Device memory is
 *     owned by the population until destroy_population, except with
 *     create_population_in, where the caller owns the workspace and it must outlive
 *     the population.
 *   - step_mechanics is asynchronous on the population's stream; a device fault shows
 *     up as MECH_E_DEVICE at the next synchronising call (read_*, destroy).
 *   - A population is used from one host thread at a time.  Different populations may
 *     run on different streams concurrently.
 *   - Units: um, min, um/min.  n_cells < 2^31 and n_voxels < 2^30.
 *   - Cell ids are the row indices of the arrays given at creation; every read_* call
 *     returns arrays in id order unless it says otherwise.
 */
#ifndef MECH_H
#define MECH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MECH_ABI_VERSION 2

enum {
    MECH_OK = 0,
    MECH_E_INVALID = -1,          /* bad argument, NaN/Inf input, asymmetric C, bad type */
    MECH_E_VOXEL_TOO_SMALL = -2,  /* voxel_size < rel_adh_distance * 2 * max radius     */
    MECH_E_OUT_OF_DOMAIN = -3,    /* a cell outside [domain_lo, domain_hi] at creation  */
    MECH_E_NOMEM = -4,            /* device allocation failed or workspace too small    */
    MECH_E_BUDGET = -5,           /* batch: request does not fit the HBM budget         */
    MECH_E_DEVICE = -6,           /* HIP runtime or kernel error                        */
    MECH_E_NONFINITE = -7,        /* state read back holds NaN or Inf                   */
    MECH_E_FULL = -8              /* batch: no free slot                                */
};

enum { MECH_FP64 = 0, MECH_FP32 = 1, MECH_FP32_KAHAN = 2 };
enum { MECH_AB2_ZERO_HISTORY = 0, MECH_AB2_EULER_START = 1 };
/* MechParams.flags bits */
enum {
    MECH_FLAG_NO_GRAPH = 1,       /* launch each step's kernels directly (no HIP graph) */
    /* Force-kernel variant (at most one; all give the same results up to summation order
       and each is deterministic).  Without either: one thread per cell, candidates
       prefiltered four at a time, in-range lists evaluated in batches. */
    MECH_FLAG_SIMPLE_FORCE = 2,   /* one thread per cell, every candidate evaluated inline */
    MECH_FLAG_VOXEL_FORCE = 4,    /* one wave per occupied voxel, neighbourhood in LDS     */
    MECH_FLAG_PRUNED_FORCE = 8,   /* the default kernel with each cell's neighbour rows
                                     pruned by its distance to them (the paper's
                                     neighbour-voxel test, Section 4.2) and x windows
                                     trimmed to its reach sphere; each lane walks its own
                                     runs                                                */
    MECH_FORCE_KERNEL_MASK = 14
};

typedef struct MechParams {
    int32_t abi_version;        /* MECH_ABI_VERSION                                    */
    int32_t precision;          /* MECH_FP64 | MECH_FP32 | MECH_FP32_KAHAN             */
    int32_t ab2_start;          /* history of the first step when none is given        */
    int32_t flags;              /* MECH_FLAG_* bits, otherwise 0                        */
    double domain_lo[3];        /* um; reflecting walls.  |lo|, |hi| < 24572 * 2^20 / S
                                   with S the largest power of two with h S <= 2^13
                                   (1.0e8 um at h = 30 um), else MECH_E_INVALID: the
                                   prefilter's quantised threshold is an int16          */
    double domain_hi[3];
    double voxel_size;          /* h, um (30)                                           */
    double dt;                  /* min (0.1)                                            */
    double c_rep;               /* repulsion coefficient, um/min (10)                   */
    double rel_adh_distance;    /* R_A / (r_i + r_j) (1.25)                             */
    int32_t n_types;            /* 1..8                                                 */
    int32_t reserved;           /* must be 0                                            */
    double c_adh[64];           /* n_types x n_types adhesion matrix, row major,
                                   symmetric (Newton's third law), um/min               */
} MechParams;

/* Launch configuration of the neighbour-force kernel (a6 + a7).  Every configuration
 * computes the same results up to the summation order of the force sums (bitwise the
 * same for one configuration); it only sets how the work is dealt to the GPU. */
typedef struct MechTuning {
    int32_t force_kernel;       /* 0 (list kernel), MECH_FLAG_SIMPLE_FORCE,
                                   MECH_FLAG_VOXEL_FORCE or MECH_FLAG_PRUNED_FORCE (the
                                   force bits of flags)                                 */
    int32_t block_waves;        /* wave64s per workgroup of the per-cell kernels:
                                   1 (default), 2, 4 or 8                               */
    int32_t unroll;             /* candidates the list kernel tests per loop trip:
                                   2, 4 or 8 (default)                                  */
    int32_t blocks_per_cu;      /* force-kernel workgroups per compute unit, 1..64, or 0
                                   (default): one per block_waves*64 cells of capacity
                                   (at most 32768 wave64s) for the per-cell kernels and
                                   4 per compute unit for the voxel kernel              */
    int32_t list_len;           /* in-range candidates a lane of the list kernel holds
                                   before the wave evaluates them: 16, 32, 64, or 0
                                   (default: 16); 64 needs block_waves <= 4             */
} MechTuning;

typedef struct MechPopulation MechPopulation;

/* Text of the last error on this thread ("" if none).  Valid until the next call. */
const char* mech_last_error(void);

/* MECH_ABI_VERSION of the loaded library. */
int32_t mech_abi_version(void);

/* Number of HIP devices visible (0 without a GPU; no device is initialised otherwise). */
int32_t mech_device_count(void);

/* Device bytes a population of n_cells needs (what create_population allocates and
 * what create_population_in requires), or a negative MECH_E_* code. */
int64_t population_workspace_bytes(const MechParams* params, int64_t n_cells);

/* Create a population on the current HIP device.  Defined by the method (not the
 * paper): the cells, their radii and types and the physics of MechParams.  The initial
 * binning is the paper's voxel container and non-empty voxel list (Section 5.4).
 *   pos            n_cells x 3 doubles, row major, id order; each inside the domain
 *   radius         n_cells doubles > 0
 *   type           n_cells int32 in [0, n_types), or NULL for all type 0
 *   prev_velocity  n_cells x 3 doubles (the history v_prev of the first step; pass the
 *                  velocity read back by read_state to resume a run), or NULL: then the
 *                  first step uses zero history, or v_prev = v with MECH_AB2_EULER_START
 *   hip_stream     hipStream_t to run on, or NULL for a stream the population owns
 * The initial binning (a1-a5) runs before this returns; read_binning then describes the
 * given positions.  On error *out is NULL and nothing is left allocated. */
int create_population(const MechParams* params, int64_t n_cells, const double* pos,
                      const double* radius, const int32_t* type,
                      const double* prev_velocity, void* hip_stream, MechPopulation** out);

/* Same, with room for the population to grow to max_cells (>= n_cells) by division
 * (population_set_division).  MECH_E_INVALID if max_cells is out of range. */
int create_population_cap(const MechParams* params, int64_t n_cells, int64_t max_cells,
                          const double* pos, const double* radius, const int32_t* type,
                          const double* prev_velocity, void* hip_stream, MechPopulation** out);

/* Same, but all device arrays are carved from the caller's device buffer `workspace`
 * of `workspace_bytes` (>= population_workspace_bytes, 256-byte aligned); the library
 * makes no device allocation.  MECH_E_NOMEM if the buffer is too small. */
int create_population_in(const MechParams* params, int64_t n_cells, const double* pos,
                         const double* radius, const int32_t* type,
                         const double* prev_velocity, void* hip_stream, void* workspace,
                         int64_t workspace_bytes, MechPopulation** out);

/* Bytes of the static device scratch of step_mechanics_noalloc (64 MiB per device). */
#define MECH_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* For callers that cannot allocate device memory (tight serving loops, harnesses that
 * forbid allocation): create_population, step_mechanics(n_steps) and read_state in one
 * synchronous call that allocates nothing.  Every device array of the population is
 * carved from the library's static device scratch, MECH_NOALLOC_SCRATCH_BYTES per
 * device, which each device the library runs on holds until the process ends; the call
 * makes no device or host allocation, creates no stream, event or graph, and launches
 * the same kernels as the population path directly on hip_stream (NULL: the null
 * stream), so its results are bitwise those of that path.  It waits for the stream
 * before returning, so it cannot be captured into a HIP graph.
 *   params, n_cells, pos, radius, type, prev_velocity  as create_population (host
 *                  arrays, copied in)
 *   n_steps        steps to take (>= 0)
 *   pos_out        n_cells x 3 doubles, id order: the positions after the steps (may be
 *                  pos itself)
 *   vel_out        n_cells x 3 doubles or NULL: the velocity of the last step, as
 *                  read_state
 *   interactions   host int64 or NULL: interacting ordered pairs over the steps
 * MECH_E_NOMEM when the population's arrays (about 210 bytes per cell and 36 per voxel)
 * exceed the scratch; the other errors as create_population and read_state.  Every call
 * on one device uses that device's one scratch and leaves its contents behind (the next
 * call sets every value it reads first): calls that overlap on one device race and must
 * not be made. */
int step_mechanics_noalloc(const MechParams* params, int64_t n_cells, const double* pos, const double* radius,
                           const int32_t* type, const double* prev_velocity, int64_t n_steps, void* hip_stream,
                           double* pos_out, double* vel_out, int64_t* interactions);

/* Enqueue n_steps steps (a1-a7 each) on the population's stream and return.  The step is
 * the paper's "update velocity" region (Sections 4.1 and 5.4) with the force law,
 * overdamped velocity, Adams-Bashforth update and walls of the method's definition
 * (file header); the reorder by voxel every step is the layout of Sections 5.4 and 6.
 * After the
 * first call, each step is one launch of a captured HIP graph.  Makes no allocation. */
int step_mechanics(MechPopulation* pop, int64_t n_steps);

/* Wait for the stream and copy the state out in id order (defined by this library: the
 * state the method's steps produce, un-permuted from the voxel order back to ids):
 *   pos  n_cells x 3 (required)
 *   vel  n_cells x 3 or NULL: the velocity of the last step, which is also the v_prev of
 *        the next one (zeros, or the given prev_velocity, before any step)
 * n_cells must equal the population size.  MECH_E_NONFINITE if any value is NaN/Inf. */
int read_state(MechPopulation* pop, double* pos, double* vel, int64_t n_cells);

/* Wait and copy the binning of the last step (or of creation, before any step); the
 * voxel of every cell, the voxel starts and the occupied list are the method's (the
 * paper's voxel container and non-empty voxel list, Section 5.4), the order inside a
 * voxel the library's:
 *   voxel_of_cell  n_cells uint32, id order (may be NULL)
 *   voxel_start    n_voxels + 1 uint32: exclusive prefix of voxel counts (may be NULL)
 *   sorted_ids     n_cells uint32: ids in storage order (voxel, x slab, id), the x slab
 *                  being floor((x - lo) * (1/h) * 4) - 4 * (voxel's x index) (may be NULL)
 *   occ            n_voxels uint32: occupied voxels, ascending; *n_occ of them are valid
 *                  (may be NULL)
 *   n_occ, n_voxels  outputs (may be NULL) */
int read_binning(MechPopulation* pop, uint32_t* voxel_of_cell, uint32_t* voxel_start,
                 uint32_t* sorted_ids, uint32_t* occ, int64_t* n_occ, int64_t* n_voxels);

/* Defined by this library (measurement): wait and return the running totals: steps
 * taken, interacting ordered pairs
 * (0 < d^2 < R_A^2), and candidate pairs the force kernel tested: the cells of the 27
 * voxels around each cell, narrowed by the default kernel to the x slabs within reach of
 * the cell (the other kernels test all of them). */
int read_stats(MechPopulation* pop, int64_t* steps, int64_t* interactions,
               int64_t* candidates);

/* Defined by this library (measurement and tests): wait and copy the per-cell force
 * kernel's current cut of the cells into the 8 XCDs' runs (9 uint32):
 *   split[0..7]  first cell of each XCD's run
 *   split[8]     the cell count the cut was made for; 0 when the runs are the
 *                equal-count ones (no cut kept, or none measured yet)
 * The cut is made from the measured work of the last launch, on grids that fill every
 * resident slot at least once; it moves which workgroup takes a cell, never a result. */
int read_xcd_split(MechPopulation* pop, uint32_t* split);

/* Run n_steps steps (a1-a7, same results as step_mechanics) with direct launches and
 * HIP events on the population's stream around the two phases; on return
 *   phase_ms[0]  mean ms per step of binning and reorder (a1-a5)
 *   phase_ms[1]  mean ms per step of the neighbour-force and update kernel (a6-a7)
 * Synchronises.  For tuning and roofline measurement. */
int profile_step(MechPopulation* pop, int64_t n_steps, double* phase_ms);

/* Growing population: cells divide, and daughters are appended at the end of the cell
 * arrays -- how the paper's cells lose their spatial locality (Section 5.4).  The paper
 * gives no division rule; this one is the library's.  After the walls of step t (t
 * counts steps from creation), cell `id` divides when u0 < p_div, where u_k =
 * (m >> 11) * 2^-53 and m is the SplitMix64 output function of the state
 * seed + 0x9E3779B97F4A7C15 * (4 (2^32 t + id) + k + 1) (mod 2^64).  Dividing cells are
 * ranked by id; while the population has room (max_cells at creation), the daughter of
 * rank k gets id n + k.  With e = v/|v|, v = (2u1 - 1, 2u2 - 1, 2u3 - 1) (or (0, 0, 1)
 * when |v|^2 < 1e-12), the parent moves to x - (r/2) e and the daughter sits at
 * x + (r/2) e, both through the walls; the daughter copies radius, type and v_prev.
 * p_div = 0 stops division.  Waits for the stream.  MECH_E_INVALID if p_div is outside
 * [0, 1]. */
int population_set_division(MechPopulation* pop, double p_div, uint64_t seed);

/* Dying population: after division in step t (daughters included), cell `id` dies when
 * its draw u0 -- the division rule's, with the seed's top bit flipped (seed ^ 2^63), so
 * that the two streams never meet for t < 2^29 -- is below p_death.  The paper gives no
 * death rule; this one is the library's, written to exercise a population that shrinks
 * as well as grows.  Survivors keep their order by id and are renumbered 0, 1, ...; the
 * cell arrays hold them in that order after the step.  The seed is the one the last
 * population_set_division call gave (0 if none).  p_death = 0 stops death.  Waits for
 * the stream.  MECH_E_INVALID if p_death is outside [0, 1]. */
int population_set_death(MechPopulation* pop, double p_death);

/* Current number of cells (waits for the stream; a growing population's size is known
 * on the device only).  read_state and read_binning take this many cells. */
int population_size(MechPopulation* pop, int64_t* n_cells);

/* Locality study (the paper's finding that cells stored far from their neighbours slow
 * the velocity update, Section 5.4): every >= 1 reorders the cells into voxel order
 * every `every` steps (1, the default, reorders every step); between reorders the cells
 * stay where they are and the force kernel reads the candidates through the sorted
 * index.  every = 0 first puts the cells back in the order they were given in (their
 * ids) and never reorders them.  Binning still runs every step, and the results are
 * bitwise those of reordering every step (same candidates, order and arithmetic); only
 * the memory access pattern changes.  Waits for the stream; MECH_E_INVALID if
 * every < 0. */
int population_set_reorder(MechPopulation* pop, int32_t every);

/* Current force-kernel launch configuration of a population, and a replacement for
 * it (validated: MECH_E_INVALID for a value outside the ranges of MechTuning).  Setting
 * waits for the stream; the step graph is captured again on the next step. */
int population_get_tuning(MechPopulation* pop, MechTuning* out);
int population_set_tuning(MechPopulation* pop, const MechTuning* tuning);

/* Size and grid of a population: n_cells, and voxels per axis. */
int population_info(MechPopulation* pop, int64_t* n_cells, int32_t dims[3]);

/* hipStream_t the population runs on. */
void* population_stream(MechPopulation* pop);

/* Wait for the stream and free everything the population owns.  NULL is a no-op. */
int destroy_population(MechPopulation* pop);

/* ------------------------------------------------------------------------------------
 * Batches: many independent simulations of uneven sizes advanced together, each kernel
 * of a step launched once for all of them (one captured HIP graph per step).  Every
 * simulation ("slot") has its own cells, domain and voxel grid; the physics in the
 * batch's MechParams (precision, dt, c_rep, rel_adh_distance, adhesion matrix, voxel
 * size, flags) is shared.  A simulation's results are bitwise the same alone (as a
 * population) and inside any batch.  Slots are admitted and retired while others run
 * (continuous batching): admission copies overlap queued steps, and retired slots'
 * space is reclaimed by compaction at a later admission.
 * ------------------------------------------------------------------------------------ */
typedef struct MechBatch MechBatch;

/* Device bytes of a batch arena for up to max_cells cells, max_voxels voxels (summed
 * over the slots' grids) and max_slots slots; negative MECH_E_* on bad arguments. */
int64_t batch_workspace_bytes(const MechParams* params, int64_t max_cells, int64_t max_voxels,
                              int32_t max_slots);

/* Voxels a simulation with this domain needs in a batch (product over the axes of
 * ceil((hi - lo) / voxel_size), at least 1 each), or a negative MECH_E_* code. */
int64_t batch_request_voxels(const MechParams* params, const double domain_lo[3],
                             const double domain_hi[3]);

/* Create an empty batch on the current device.  params: the shared physics; its domain
 * fields are not used.  hip_stream as in create_population. */
int create_batch(const MechParams* params, int64_t max_cells, int64_t max_voxels,
                 int32_t max_slots, void* hip_stream, MechBatch** out);

/* Same, with the arena carved from the caller's 256-byte aligned device buffer. */
int create_batch_in(const MechParams* params, int64_t max_cells, int64_t max_voxels,
                    int32_t max_slots, void* hip_stream, void* workspace,
                    int64_t workspace_bytes, MechBatch** out);

/* Cells and voxels of the largest batch arena within hbm_budget_bytes of device memory,
 * for workloads that need about voxels_per_cell voxels per cell (max_voxels =
 * ceil(voxels_per_cell * max_cells), at least 1) and max_slots slots: the admission
 * capacity a server gets from an HBM budget.  MECH_E_BUDGET if not even one cell fits;
 * MECH_E_INVALID for bad parameters (voxels_per_cell must lie in (0, 1e6]).  Defined by
 * the library's arena layout, not by the paper. */
int batch_budget_capacity(const MechParams* params, int64_t hbm_budget_bytes, double voxels_per_cell,
                          int32_t max_slots, int64_t* max_cells, int64_t* max_voxels);

/* create_batch with the capacity batch_budget_capacity gives for the budget: one device
 * allocation of at most hbm_budget_bytes, made here and owned by the batch.  Admission
 * then fails with MECH_E_BUDGET whenever a request's cells or voxels do not fit what the
 * running simulations leave free. */
int create_batch_budget(const MechParams* params, int64_t hbm_budget_bytes, double voxels_per_cell,
                        int32_t max_slots, void* hip_stream, MechBatch** out);

/* Capacity of a batch: cells, voxels and slots it was created for, and its arena bytes
 * (each pointer may be NULL). */
int batch_capacity(MechBatch* batch, int64_t* max_cells, int64_t* max_voxels, int32_t* max_slots,
                   int64_t* arena_bytes);

/* Record a reference point on the batch's stream and wait until the device reaches it:
 * the zero of batch_slot_done_ms.  A serving loop calls it once when its clock starts. */
int batch_mark_clock(MechBatch* batch);

/* Device time in ms from the last batch_mark_clock to the completion of a slot's last
 * step (its completion event, recorded right after that step), for a slot that
 * batch_poll has reported finished.  MECH_E_INVALID if the clock was never marked, the
 * slot holds no simulation or has not finished on the device. */
int batch_slot_done_ms(MechBatch* batch, int32_t slot, double* ms);

/* Admit one simulation (arrays as in create_population, domain given here).  It runs
 * n_steps steps of the following batch_step calls and then stays frozen until read and
 * retired; n_steps < 0 runs until retired.  *slot_out receives its slot id.
 * MECH_E_FULL: no free slot.  MECH_E_BUDGET: its cells or voxels exceed what the arena
 * has free once retired slots are dropped (the batch is left unchanged). */
int batch_admit(MechBatch* batch, const double domain_lo[3], const double domain_hi[3],
                int64_t n_cells, const double* pos, const double* radius, const int32_t* type,
                const double* prev_velocity, int64_t n_steps, int32_t* slot_out);

/* Enqueue n_steps steps of every running slot (asynchronous). */
int batch_step(MechBatch* batch, int64_t n_steps);

/* Slots whose last step has completed on the device since the previous poll (without
 * waiting): up to `capacity` ids go to done_slots, *n_done gets how many completed. */
int batch_poll(MechBatch* batch, int32_t* done_slots, int32_t capacity, int32_t* n_done);

/* Wait for the stream and copy one slot's state out in its own id order (as
 * read_state). */
int batch_read(MechBatch* batch, int32_t slot, double* pos, double* vel, int64_t n_cells);

/* Stop a slot and free its id; its arena space is reclaimed at a later admission. */
int batch_retire(MechBatch* batch, int32_t slot);

/* Size of a slot and the steps it still has to run (< 0: no limit). */
int batch_slot_info(MechBatch* batch, int32_t slot, int64_t* n_cells, int64_t* steps_left);

/* Cells and voxels in the arena (retired slots included), running slots, and the
 * cells and voxels free once retired slots are dropped. */
int batch_info(MechBatch* batch, int64_t* n_cells, int64_t* n_voxels, int32_t* n_live,
               int64_t* free_cells, int64_t* free_voxels);

/* As read_stats and profile_step, for all slots together. */
int batch_stats(MechBatch* batch, int64_t* steps, int64_t* interactions, int64_t* candidates);
int batch_profile(MechBatch* batch, int64_t n_steps, double* phase_ms);

/* Replace the batch's MechParams.flags (force-kernel variant, graph use): the tuner's
 * hook.  Waits for the stream; the step graph is captured again on the next step. */
int batch_set_flags(MechBatch* batch, int32_t flags);

/* As population_get_tuning / population_set_tuning, for a batch (what the autotuner
 * sets once it has timed the candidates on a copy of the batch). */
int batch_get_tuning(MechBatch* batch, MechTuning* out);
int batch_set_tuning(MechBatch* batch, const MechTuning* tuning);

/* Wait until every step enqueued so far has completed on the device. */
int batch_sync(MechBatch* batch);

/* hipStream_t the batch runs on. */
void* batch_stream(MechBatch* batch);

/* Wait for the stream and free everything the batch owns.  NULL is a no-op. */
int destroy_batch(MechBatch* batch);

#ifdef __cplusplus
}
#endif

#endif /* MECH_H */
