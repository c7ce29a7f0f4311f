/* A plain C driver of the two oracles (mech_oracle.c, diffusion_oracle.c), built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by test_sanitizers.py and run on the
 * CPU: every oracle function on small seeded inputs, with ragged sizes, a coincident
 * pair, a full-capacity division and a one-voxel mesh.  Exit status 0 and no sanitizer
 * report is the pass.  The struct layouts repeat the oracles' own (test infrastructure
 * only). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double lo[3], hi[3];
    double h, dt, c_rep, alpha;
    int32_t n_types;
    int32_t pad_;
    double c_adh[64];
} OracleParams;

typedef struct {
    int32_t dims[3];
    int32_t n_substrates;
    double dx;
    double dt;
    double diffusion[16];
    double decay[16];
} DiffOracleParams;

int32_t oracle_grid_dims(const OracleParams* p, int32_t dims[3]);
int32_t oracle_bin(const OracleParams* p, int64_t n, const double* pos, uint32_t* vid, uint32_t* voxel_start,
                   uint32_t* sorted_ids, uint32_t* occ, int64_t* n_occ);
int32_t oracle_velocity_allpairs(const OracleParams* p, int64_t n, const double* pos, const double* radius,
                                 const int32_t* type, int32_t precision, double* vel, int64_t* interactions);
int32_t oracle_velocity_voxel(const OracleParams* p, int64_t n, const double* pos, const double* radius,
                              const int32_t* type, int32_t precision, double* vel, int64_t* interactions,
                              int64_t* candidates);
int32_t oracle_run(const OracleParams* p, int64_t n, double* pos, const double* radius, const int32_t* type,
                   double* vprev, int64_t steps, int32_t precision, int32_t euler_first, int32_t allpairs,
                   int64_t* per_step, int64_t* interactions, int64_t* candidates);
int32_t oracle_velocity_sampled(const OracleParams* p, int64_t n, const double* pos, const double* radius,
                                const int32_t* type, int32_t precision, int64_t n_sample, const int64_t* ids,
                                double* vel, int64_t* interactions);
int32_t oracle_divide(const OracleParams* p, int64_t n, int64_t capacity, double* pos, double* radius,
                      int32_t* type, double* vprev, uint64_t seed, int64_t t, double p_div, int64_t* n_out);
int32_t oracle_die(int64_t n, double* pos, double* radius, int32_t* type, double* vprev, uint64_t seed, int64_t t,
                   double p_death, int64_t* n_out);
float oracle_sum_f32(const float* x, int64_t n, int32_t kahan);
int32_t oracle_diffusion_step(const DiffOracleParams* p, double* rho, int64_t n_steps);
int32_t oracle_diffusion_sweep(const DiffOracleParams* p, double* rho, int32_t axis);
int32_t oracle_gradients(const DiffOracleParams* p, const double* rho, double* grad);

static uint64_t rs = 88172645463325252ull;
static double urand(void)
{
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) * 0x1p-53;
}

static int fails = 0;
#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);         \
            ++fails;                                                   \
        }                                                              \
    } while (0)

static void mechanics(int64_t n, int precision, int two_types)
{
    OracleParams p;
    memset(&p, 0, sizeof p);
    for (int a = 0; a < 3; ++a) {
        p.lo[a] = -50.0;
        p.hi[a] = 47.0;   /* the grid overruns hi */
    }
    p.h = 30.0;
    p.dt = 0.1;
    p.c_rep = 10.0;
    p.alpha = 1.25;
    p.n_types = two_types ? 2 : 1;
    p.c_adh[0] = 0.4;
    p.c_adh[1] = p.c_adh[2] = 0.1;
    p.c_adh[3] = 0.4;
    int32_t dims[3];
    CHECK(oracle_grid_dims(&p, dims) == 0);
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    const int64_t cap = n + n / 2 + 1;
    double* pos = calloc((size_t)cap * 3, sizeof(double));
    double* rad = calloc((size_t)cap, sizeof(double));
    int32_t* typ = calloc((size_t)cap, sizeof(int32_t));
    double* vp = calloc((size_t)cap * 3, sizeof(double));
    double* vel = calloc((size_t)(n > 3 ? n : 3) * 3, sizeof(double));   /* also the 3 sampled rows */
    uint32_t* vid = calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    uint32_t* start = calloc((size_t)V + 1, sizeof(uint32_t));
    uint32_t* ids = calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    uint32_t* occ = calloc((size_t)V, sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) pos[3 * i + a] = -50.0 + 97.0 * urand();
        rad[i] = 6.0 + 5.0 * urand();
        typ[i] = two_types ? (int32_t)(urand() < 0.5) : 0;
    }
    if (n >= 2)
        for (int a = 0; a < 3; ++a) pos[3 + a] = pos[a];   /* a coincident pair */
    if (n >= 1) pos[0] = p.hi[0];                        /* a cell on the upper wall */
    int64_t m = 0, inter = 0, cand = 0, inter2 = 0;
    CHECK(oracle_bin(&p, n, pos, vid, start, ids, occ, &m) == 0);
    CHECK(start[V] == (uint32_t)n && m <= V);
    CHECK(oracle_velocity_voxel(&p, n, pos, rad, typ, precision, vel, &inter, &cand) == 0);
    CHECK(oracle_velocity_allpairs(&p, n, pos, rad, typ, precision, vel, &inter2) == 0);
    CHECK(inter == inter2);
    int64_t sample[3] = {0, n > 1 ? n - 1 : 0, n / 2};
    if (n > 0) CHECK(oracle_velocity_sampled(&p, n, pos, rad, typ, precision, 3, sample, vel, &inter2) == 0);
    int64_t per[3];
    CHECK(oracle_run(&p, n, pos, rad, typ, vp, 3, precision, 1, 0, per, &inter, &cand) == 0);
    int64_t nn = n;
    CHECK(oracle_divide(&p, nn, cap, pos, rad, typ, vp, 7, 0, 0.9, &nn) == 0);
    CHECK(nn >= n && nn <= cap);
    CHECK(oracle_die(nn, pos, rad, typ, vp, 7, 0, 0.3, &nn) == 0);
    CHECK(nn >= 0 && nn <= cap);
    free(pos);
    free(rad);
    free(typ);
    free(vp);
    free(vel);
    free(vid);
    free(start);
    free(ids);
    free(occ);
}

static void diffusion(int nx, int ny, int nz, int ns)
{
    DiffOracleParams p;
    memset(&p, 0, sizeof p);
    p.dims[0] = nx;
    p.dims[1] = ny;
    p.dims[2] = nz;
    p.n_substrates = ns;
    p.dx = 20.0;
    p.dt = 0.05;
    for (int s = 0; s < ns; ++s) {
        p.diffusion[s] = 1e3 * (s + 1);
        p.decay[s] = 0.1 * s;
    }
    const size_t V = (size_t)nx * ny * nz;
    double* rho = malloc(V * ns * sizeof(double));
    double* grad = malloc(3 * V * ns * sizeof(double));
    for (size_t k = 0; k < V * ns; ++k) rho[k] = urand();
    CHECK(oracle_diffusion_step(&p, rho, 2) == 0);
    for (int a = 0; a < 3; ++a) CHECK(oracle_diffusion_sweep(&p, rho, a) == 0);
    CHECK(oracle_gradients(&p, rho, grad) == 0);
    free(rho);
    free(grad);
}

int main(void)
{
    const int64_t sizes[] = {0, 1, 2, 37, 300};
    for (int k = 0; k < 5; ++k)
        for (int prec = 0; prec < 3; ++prec) mechanics(sizes[k], prec, k & 1);
    float xs[100];
    for (int k = 0; k < 100; ++k) xs[k] = (float)urand();
    (void)oracle_sum_f32(xs, 100, 1);
    (void)oracle_sum_f32(xs, 0, 0);
    diffusion(1, 1, 1, 1);
    diffusion(7, 5, 3, 2);
    diffusion(1, 9, 1, 3);
    diffusion(16, 1, 4, 1);
    if (fails) return 1;
    printf("oracle sanitized ok\n");
    return 0;
}
