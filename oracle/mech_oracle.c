/*
 * mech_oracle.c -- plain, slow CPU oracle for the agent-mechanics step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg load this library; the product path (the HIP library) never does and
 * shares no code with it.
 *
 * What it computes (one step, all FP64 unless the FP32 variant is asked for):
 *   1. Grid: n_a = ceil((hi_a - lo_a) / h) voxels per axis, anchored at lo, edge h.
 *      Voxels are numbered x fastest: vid = kx + nx*(ky + ny*kz).  The paper's
 *      voxel-parallel update walks a linear container of mechanics voxels (Section 5.4,
 *      the voxel-based update-velocity listing); the x-fastest numbering is our reading.
 *   2. Binning: k_a = clamp(floor((x_a - lo_a) * (1/h)), 0, n_a - 1); a counting sort
 *      by voxel id, stable in cell id, lists the cells voxel by voxel (ascending voxel
 *      id) and inside a voxel by ascending cell id.  Only occupied voxels are listed in
 *      `occ` (the paper's non-empty voxel list, Section 5.4).
 *   3. Velocity (overdamped: velocity = sum of pair forces, unit mobility), gathered
 *      over the 27 voxels around the cell's own voxel, dz outermost, then dy, then dx,
 *      each voxel's cells by ascending id:
 *        delta = x_i - x_j, d2 = |delta|^2, R = r_i + r_j, R_A = alpha * R
 *        a pair interacts when 0 < d2 < R_A*R_A
 *        w = c_rep (1 - d/R)^2 [d < R]  -  C[t_i][t_j] (1 - d/R_A)^2
 *        v_i += (w / d) * delta
 *      Repulsion pushes i away from j, adhesion pulls it towards j.
 *   4. Two-step Adams-Bashforth: x <- x + dt (1.5 v - 0.5 v_prev).  With the Euler
 *      start, the first step of a run takes v_prev = v (a plain forward-Euler step).
 *   5. Reflecting walls on cell centres, per axis: x < lo -> 2lo - x, x > hi -> 2hi - x,
 *      then clamp to [lo, hi].  v_prev is not touched by a reflection.
 *   6. v_prev <- v.
 *
 * The paper is a CPU performance study and prints none of these equations; the force
 * law, the overdamped velocity, the two-step Adams-Bashforth update, the 30 um voxel
 * and the walls are the method's definition as this project takes it.  The paper's part
 * is the hot region itself ("update velocity", Sections 4 and 5.4) and its traversal
 * lessons: compute cells voxel by voxel in mesh order and skip empty voxels (Section
 * 5.4) -- which this oracle also follows, since it is the algorithm being checked.
 *
 * FP32 variant (an approximation): positions and radii are rounded to float once per
 * step and the pair arithmetic of step 3 runs in float, each operation of the written
 * expressions rounded on its own (d2 = (dx*dx + dy*dy) + dz*dz, no fused forms); the
 * force sum is plain float or Kahan-compensated per component (Kahan 1965; the result
 * is the running sum, its correction term is not added back), and the update in step 4
 * runs in double on the float velocity; v_prev holds the float velocity.
 *
 * Everything is compiled with -ffp-contract=off, so every result is the IEEE value of the
 * expression as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double lo[3], hi[3];
    double h, dt, c_rep, alpha;
    int32_t n_types;
    int32_t pad_;
    double c_adh[64];          /* n_types x n_types, row major */
} OracleParams;

enum { OR_FP64 = 0, OR_FP32 = 1, OR_FP32_KAHAN = 2 };

/* ------------------------------------------------------------------ grid + binning */

int32_t oracle_grid_dims(const OracleParams* p, int32_t dims[3])
{
    for (int a = 0; a < 3; ++a) {
        double span = p->hi[a] - p->lo[a];
        if (!(span >= 0.0) || !(p->h > 0.0)) return -1;
        long n = (long)ceil(span / p->h);
        if (n < 1) n = 1;
        dims[a] = (int32_t)n;
    }
    return 0;
}

/* Voxel id of a position. */
static int64_t voxel_of(const OracleParams* p, const int32_t dims[3], double inv_h, const double* x)
{
    int64_t k[3];
    for (int a = 0; a < 3; ++a) {
        double f = floor((x[a] - p->lo[a]) * inv_h);
        int64_t ka = (int64_t)f;
        if (f < 0.0) ka = 0;
        if (ka > dims[a] - 1) ka = dims[a] - 1;
        k[a] = ka;
    }
    return k[0] + (int64_t)dims[0] * (k[1] + (int64_t)dims[1] * k[2]);
}

/* vid[n]; voxel_start[V+1]; sorted_ids[n]; occ[V] (first *n_occ used). */
int32_t oracle_bin(const OracleParams* p, int64_t n, const double* pos, uint32_t* vid,
                   uint32_t* voxel_start, uint32_t* sorted_ids, uint32_t* occ,
                   int64_t* n_occ)
{
    int32_t dims[3];
    if (oracle_grid_dims(p, dims)) return -1;
    int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    double inv_h = 1.0 / p->h;
    uint32_t* cursor = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)V + 1));
    if (!cursor) return -2;
    for (int64_t i = 0; i < n; ++i) vid[i] = (uint32_t)voxel_of(p, dims, inv_h, pos + 3 * i);
    /* counts per voxel, then exclusive prefix */
    memset(voxel_start, 0, sizeof(uint32_t) * ((size_t)V + 1));
    for (int64_t i = 0; i < n; ++i) voxel_start[vid[i] + 1] += 1;
    for (int64_t v = 0; v < V; ++v) voxel_start[v + 1] += voxel_start[v];
    /* placing the cells in ascending id order keeps each voxel's cells in id order */
    memcpy(cursor, voxel_start, sizeof(uint32_t) * ((size_t)V + 1));
    for (int64_t i = 0; i < n; ++i) sorted_ids[cursor[vid[i]]++] = (uint32_t)i;
    int64_t m = 0;
    for (int64_t v = 0; v < V; ++v)
        if (voxel_start[v + 1] > voxel_start[v]) occ[m++] = (uint32_t)v;
    *n_occ = m;
    free(cursor);
    return 0;
}

/* ------------------------------------------------------------------ pair terms */

/* FP64 pair term.  Returns 1 when the pair interacts (and adds its term to acc). */
static int pair_f64(const OracleParams* p, const double* xi, double ri, int ti,
                    const double* xj, double rj, int tj, double acc[3])
{
    double dx = xi[0] - xj[0], dy = xi[1] - xj[1], dz = xi[2] - xj[2];
    double d2 = dx * dx + dy * dy + dz * dz;
    double R = ri + rj;
    double RA = p->alpha * R;
    if (!(d2 > 0.0 && d2 < RA * RA)) return 0;
    double d = sqrt(d2);
    double w = 0.0;
    if (d < R) {
        double u = 1.0 - d / R;
        w += p->c_rep * u * u;
    }
    double a = 1.0 - d / RA;
    w -= p->c_adh[ti * p->n_types + tj] * a * a;
    double s = w / d;
    acc[0] += s * dx;
    acc[1] += s * dy;
    acc[2] += s * dz;
    return 1;
}

typedef struct { float s[3], c[3]; } AccF;

/* One step of a float sum: plain, or Kahan-compensated (c carries the low part lost by
 * the last addition, subtracted from the next term; the sum itself is the result). */
static void accumulate_f32(float* sum, float* c, float term, int kahan)
{
    if (kahan) {
        float y = term - *c;
        float t = *sum + y;
        *c = (t - *sum) - y;
        *sum = t;
    } else {
        *sum += term;
    }
}

/* FP32 pair term on float copies of the positions and radii. */
static int pair_f32(const OracleParams* p, const float* xi, float ri, int ti,
                    const float* xj, float rj, int tj, AccF* acc, int kahan)
{
    float dx = xi[0] - xj[0], dy = xi[1] - xj[1], dz = xi[2] - xj[2];
    float d2 = dx * dx + dy * dy + dz * dz;
    float R = ri + rj;
    float RA = (float)p->alpha * R;
    if (!(d2 > 0.0f && d2 < RA * RA)) return 0;
    float d = sqrtf(d2);
    float w = 0.0f;
    if (d < R) {
        float u = 1.0f - d / R;
        w += (float)p->c_rep * u * u;
    }
    float a = 1.0f - d / RA;
    w -= (float)p->c_adh[ti * p->n_types + tj] * a * a;
    float s = w / d;
    float term[3] = { s * dx, s * dy, s * dz };
    for (int c = 0; c < 3; ++c) accumulate_f32(&acc->s[c], &acc->c[c], term[c], kahan);
    return 1;
}

/* Sum of n floats with the same accumulator the FP32 velocity uses (test hook). */
float oracle_sum_f32(const float* x, int64_t n, int32_t kahan)
{
    float s = 0.0f, c = 0.0f;
    for (int64_t i = 0; i < n; ++i) accumulate_f32(&s, &c, x[i], kahan);
    return s;
}

/* ------------------------------------------------------------------ velocities */

/* Plain definition: every ordered pair (i, j), j ascending.  O(n^2). */
int32_t oracle_velocity_allpairs(const OracleParams* p, int64_t n, const double* pos,
                                 const double* radius, const int32_t* type,
                                 int32_t precision, double* vel, int64_t* interactions)
{
    int64_t inter = 0;
    float* pf = NULL;
    float* rf = NULL;
    if (precision != OR_FP64) {
        pf = (float*)malloc(sizeof(float) * 3 * (size_t)(n ? n : 1));
        rf = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
        if (!pf || !rf) { free(pf); free(rf); return -2; }
        for (int64_t i = 0; i < 3 * n; ++i) pf[i] = (float)pos[i];
        for (int64_t i = 0; i < n; ++i) rf[i] = (float)radius[i];
    }
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : inter)
    for (int64_t i = 0; i < n; ++i) {
        int ti = type ? type[i] : 0;
        if (precision == OR_FP64) {
            double acc[3] = { 0.0, 0.0, 0.0 };
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                inter += pair_f64(p, pos + 3 * i, radius[i], ti, pos + 3 * j, radius[j],
                                  type ? type[j] : 0, acc);
            }
            for (int c = 0; c < 3; ++c) vel[3 * i + c] = acc[c];
        } else {
            AccF acc;
            memset(&acc, 0, sizeof acc);
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                inter += pair_f32(p, pf + 3 * i, rf[i], ti, pf + 3 * j, rf[j],
                                  type ? type[j] : 0, &acc, precision == OR_FP32_KAHAN);
            }
            for (int c = 0; c < 3; ++c) vel[3 * i + c] = (double)acc.s[c];
        }
    }
    free(pf);
    free(rf);
    if (interactions) *interactions = inter;
    return 0;
}

/* The method: bin, then gather each cell's velocity from the 27 surrounding voxels.
 * vel is written in cell-id order.  candidates counts the pairs (i, j != i) visited. */
int32_t oracle_velocity_voxel(const OracleParams* p, int64_t n, const double* pos,
                              const double* radius, const int32_t* type, int32_t precision,
                              double* vel, int64_t* interactions, int64_t* candidates)
{
    int32_t dims[3];
    if (oracle_grid_dims(p, dims)) return -1;
    int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    size_t nn = (size_t)(n ? n : 1);
    uint32_t* vid = (uint32_t*)malloc(sizeof(uint32_t) * nn);
    uint32_t* start = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)V + 1));
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * nn);
    uint32_t* occ = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)V);
    float* pf = NULL;
    float* rf = NULL;
    int rc = 0;
    if (!vid || !start || !ids || !occ) { rc = -2; goto done; }
    if (precision != OR_FP64) {
        pf = (float*)malloc(sizeof(float) * 3 * nn);
        rf = (float*)malloc(sizeof(float) * nn);
        if (!pf || !rf) { rc = -2; goto done; }
        for (int64_t i = 0; i < 3 * n; ++i) pf[i] = (float)pos[i];
        for (int64_t i = 0; i < n; ++i) rf[i] = (float)radius[i];
    }
    int64_t m;
    if (oracle_bin(p, n, pos, vid, start, ids, occ, &m)) { rc = -1; goto done; }

    int64_t inter = 0, cand = 0;
    /* cells are computed voxel by voxel, in the binned (mesh) order */
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : inter, cand)
    for (int64_t s = 0; s < n; ++s) {
        int64_t i = ids[s];
        int64_t v = vid[i];
        int64_t kx = v % dims[0], ky = (v / dims[0]) % dims[1], kz = v / ((int64_t)dims[0] * dims[1]);
        int ti = type ? type[i] : 0;
        double acc[3] = { 0.0, 0.0, 0.0 };
        AccF accf;
        memset(&accf, 0, sizeof accf);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t x = kx + dx, y = ky + dy, z = kz + dz;
                    if (x < 0 || y < 0 || z < 0 || x >= dims[0] || y >= dims[1] || z >= dims[2])
                        continue;
                    int64_t u = x + (int64_t)dims[0] * (y + (int64_t)dims[1] * z);
                    for (uint32_t q = start[u]; q < start[u + 1]; ++q) {
                        int64_t j = ids[q];
                        if (j == i) continue;
                        ++cand;
                        int tj = type ? type[j] : 0;
                        if (precision == OR_FP64)
                            inter += pair_f64(p, pos + 3 * i, radius[i], ti, pos + 3 * j,
                                              radius[j], tj, acc);
                        else
                            inter += pair_f32(p, pf + 3 * i, rf[i], ti, pf + 3 * j, rf[j], tj,
                                              &accf, precision == OR_FP32_KAHAN);
                    }
                }
        for (int c = 0; c < 3; ++c)
            vel[3 * i + c] = (precision == OR_FP64) ? acc[c] : (double)accf.s[c];
    }
    if (interactions) *interactions = inter;
    if (candidates) *candidates = cand;
done:
    free(vid); free(start); free(ids); free(occ); free(pf); free(rf);
    return rc;
}

/* ------------------------------------------------------------------ integration */

static double reflect(double x, double lo, double hi)
{
    if (x < lo) x = 2.0 * lo - x;
    if (x > hi) x = 2.0 * hi - x;
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    return x;
}

/* One Adams-Bashforth step plus walls, given this step's velocity. */
int32_t oracle_integrate(const OracleParams* p, int64_t n, double* pos, const double* vel,
                         double* vprev, int32_t euler_start)
{
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            double v = vel[3 * i + c];
            double vp = euler_start ? v : vprev[3 * i + c];
            double x = pos[3 * i + c] + p->dt * (1.5 * v - 0.5 * vp);
            pos[3 * i + c] = reflect(x, p->lo[c], p->hi[c]);
            vprev[3 * i + c] = v;
        }
    return 0;
}

/* n_steps steps: velocity by the 27-voxel method (or all pairs), then integrate.
 * euler_first: the first of these steps uses the Euler start.  per_step_inter, when
 * not NULL, receives each step's interaction count. */
int32_t oracle_run(const OracleParams* p, int64_t n, double* pos, const double* radius,
                   const int32_t* type, double* vprev, int64_t n_steps, int32_t precision,
                   int32_t euler_first, int32_t allpairs, int64_t* per_step_inter,
                   int64_t* interactions, int64_t* candidates)
{
    double* vel = (double*)malloc(sizeof(double) * 3 * (size_t)(n ? n : 1));
    if (!vel) return -2;
    int64_t tot_i = 0, tot_c = 0;
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t it = 0, ct = 0;
        int32_t rc = allpairs
            ? oracle_velocity_allpairs(p, n, pos, radius, type, precision, vel, &it)
            : oracle_velocity_voxel(p, n, pos, radius, type, precision, vel, &it, &ct);
        if (rc) { free(vel); return rc; }
        oracle_integrate(p, n, pos, vel, vprev, euler_first && s == 0);
        if (per_step_inter) per_step_inter[s] = it;
        tot_i += it;
        tot_c += ct;
    }
    if (interactions) *interactions = tot_i;
    if (candidates) *candidates = tot_c;
    free(vel);
    return 0;
}

/* Velocity of a few selected cells (by id) from the 27-voxel neighbourhood, each
 * computed on its own: used to check sampled outputs of very large populations. */
int32_t oracle_velocity_sampled(const OracleParams* p, int64_t n, const double* pos,
                                const double* radius, const int32_t* type, int32_t precision,
                                int64_t n_sample, const int64_t* sample_ids, double* vel,
                                int64_t* interactions)
{
    int32_t dims[3];
    if (oracle_grid_dims(p, dims)) return -1;
    int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    size_t nn = (size_t)(n ? n : 1);
    uint32_t* vid = (uint32_t*)malloc(sizeof(uint32_t) * nn);
    uint32_t* start = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)V + 1));
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * nn);
    uint32_t* occ = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)V);
    int rc = 0;
    int64_t m;
    if (!vid || !start || !ids || !occ) { rc = -2; goto done; }
    if (oracle_bin(p, n, pos, vid, start, ids, occ, &m)) { rc = -1; goto done; }
    int64_t inter = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : inter)
    for (int64_t k = 0; k < n_sample; ++k) {
        int64_t i = sample_ids[k];
        int64_t v = vid[i];
        int64_t kx = v % dims[0], ky = (v / dims[0]) % dims[1], kz = v / ((int64_t)dims[0] * dims[1]);
        int ti = type ? type[i] : 0;
        double acc[3] = { 0.0, 0.0, 0.0 };
        AccF accf;
        memset(&accf, 0, sizeof accf);
        float xi[3] = { (float)pos[3 * i], (float)pos[3 * i + 1], (float)pos[3 * i + 2] };
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t x = kx + dx, y = ky + dy, z = kz + dz;
                    if (x < 0 || y < 0 || z < 0 || x >= dims[0] || y >= dims[1] || z >= dims[2])
                        continue;
                    int64_t u = x + (int64_t)dims[0] * (y + (int64_t)dims[1] * z);
                    for (uint32_t q = start[u]; q < start[u + 1]; ++q) {
                        int64_t j = ids[q];
                        if (j == i) continue;
                        int tj = type ? type[j] : 0;
                        if (precision == OR_FP64) {
                            inter += pair_f64(p, pos + 3 * i, radius[i], ti, pos + 3 * j,
                                              radius[j], tj, acc);
                        } else {
                            float xj[3] = { (float)pos[3 * j], (float)pos[3 * j + 1],
                                            (float)pos[3 * j + 2] };
                            inter += pair_f32(p, xi, (float)radius[i], ti, xj, (float)radius[j],
                                              tj, &accf, precision == OR_FP32_KAHAN);
                        }
                    }
                }
        for (int c = 0; c < 3; ++c)
            vel[3 * k + c] = (precision == OR_FP64) ? acc[c] : (double)accf.s[c];
    }
    if (interactions) *interactions = inter;
done:
    free(vid); free(start); free(ids); free(occ);
    return rc;
}

/* ------------------------------------------------------------------ division */

/* Growing populations (the source of the locality loss the paper studies, Section 5.4:
 * cells created by division are appended at the end of the cell vector).  The paper
 * gives no division rule; this is the one the library defines:
 *   - after the walls of step t (t counts steps from creation, from 0), cell `id`
 *     divides when u0 < p_div, with u_k = uniform(seed, id, t, k) below;
 *   - dividing cells are ranked by ascending id; the first min(D, capacity - n) of them
 *     divide (D of them drew a division), the daughter of rank k taking id n + k;
 *   - direction e = v / |v| with v = (2 u1 - 1, 2 u2 - 1, 2 u3 - 1), or (0, 0, 1) when
 *     |v|^2 < 1e-12; the parent moves to x - (r/2) e and the daughter sits at
 *     x + (r/2) e, both through the walls of step 5 of the method;
 *   - the daughter copies the parent's radius, type and v_prev.
 * uniform(seed, id, t, k) = (m >> 11) * 2^-53 where m is the output function of
 * SplitMix64 (Steele, Lea and Flood 2014, as in Vigna's reference code) applied to the
 * state seed + 0x9E3779B97F4A7C15 * (4 (2^32 t + id) + k + 1), all mod 2^64. */
uint64_t oracle_splitmix64(uint64_t state)
{
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double oracle_uniform(uint64_t seed, uint64_t id, uint64_t t, uint64_t k)
{
    uint64_t counter = 4u * ((t << 32) + id) + k + 1u;
    uint64_t m = oracle_splitmix64(seed + 0x9E3779B97F4A7C15ull * counter);
    return (double)(m >> 11) * (1.0 / 9007199254740992.0);
}

/* Arrays in id order with room for `capacity` cells; returns the new size in *n_out. */
int32_t oracle_divide(const OracleParams* p, int64_t n, int64_t capacity, double* pos,
                      double* radius, int32_t* type, double* vprev, uint64_t seed, int64_t t,
                      double p_div, int64_t* n_out)
{
    int64_t made = 0;
    for (int64_t id = 0; id < n && n + made < capacity; ++id) {
        if (!(oracle_uniform(seed, (uint64_t)id, (uint64_t)t, 0) < p_div)) continue;
        double v[3];
        for (int c = 0; c < 3; ++c)
            v[c] = 2.0 * oracle_uniform(seed, (uint64_t)id, (uint64_t)t, (uint64_t)c + 1) - 1.0;
        double l2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        double e[3] = { 0.0, 0.0, 1.0 };
        if (l2 >= 1e-12) {
            double l = sqrt(l2);
            for (int c = 0; c < 3; ++c) e[c] = v[c] / l;
        }
        int64_t q = n + made;
        double half = 0.5 * radius[id];
        for (int c = 0; c < 3; ++c) {
            double x = pos[3 * id + c];
            pos[3 * q + c] = reflect(x + half * e[c], p->lo[c], p->hi[c]);
            pos[3 * id + c] = reflect(x - half * e[c], p->lo[c], p->hi[c]);
            vprev[3 * q + c] = vprev[3 * id + c];
        }
        radius[q] = radius[id];
        type[q] = type[id];
        ++made;
    }
    *n_out = n + made;
    return 0;
}

/* Death (the other half of a dynamic population; the paper gives no rule either), after
 * division in the same step:
 *   - every cell, daughters of this step included, dies when
 *     uniform(seed XOR 2^63, id, t, 0) < p_death: the draw of division's generator with
 *     the seed's top bit flipped.  Its states differ from those of the division draws by
 *     gamma times (counter difference + 2^63), nonzero mod 2^64 for t < 2^29: the two
 *     streams never share a state;
 *   - the dead are removed and the survivors keep their order, renumbered 0, 1, ... by
 *     ascending old id, with their position, radius, type and v_prev unchanged. */
int32_t oracle_die(int64_t n, double* pos, double* radius, int32_t* type, double* vprev,
                   uint64_t seed, int64_t t, double p_death, int64_t* n_out)
{
    const uint64_t seed_d = seed ^ 0x8000000000000000ull;
    int64_t kept = 0;
    for (int64_t id = 0; id < n; ++id) {
        if (oracle_uniform(seed_d, (uint64_t)id, (uint64_t)t, 0) < p_death) continue;
        if (kept != id) {
            for (int c = 0; c < 3; ++c) {
                pos[3 * kept + c] = pos[3 * id + c];
                vprev[3 * kept + c] = vprev[3 * id + c];
            }
            radius[kept] = radius[id];
            type[kept] = type[id];
        }
        ++kept;
    }
    *n_out = kept;
    return 0;
}

/* ------------------------------------------------------------------ threads */

int32_t oracle_set_threads(int32_t t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}
