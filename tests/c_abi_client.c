/* A plain C client of libmech.so: builds against include/mech.h and include/microenv.h
 * alone (no Python, no torch types) and exercises the calls that need no GPU.  Run by
 * test_abi.py, and by test_sanitizers.py against a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mech.h"
#include "microenv.h"

static int fails = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond);     \
            ++fails;                                                  \
        }                                                             \
    } while (0)

int main(void)
{
    MechParams p;
    memset(&p, 0, sizeof p);
    p.abi_version = MECH_ABI_VERSION;
    p.precision = MECH_FP32_KAHAN;
    for (int a = 0; a < 3; ++a) {
        p.domain_lo[a] = -100.0;
        p.domain_hi[a] = 100.0;
    }
    p.voxel_size = 30.0;
    p.dt = 0.1;
    p.c_rep = 10.0;
    p.rel_adh_distance = 1.25;
    p.n_types = 1;
    p.c_adh[0] = 0.4;

    CHECK(mech_abi_version() == MECH_ABI_VERSION);
    const int64_t one = population_workspace_bytes(&p, 1000);
    const int64_t two = population_workspace_bytes(&p, 2000);
    CHECK(one > 0 && two > one);
    CHECK(batch_request_voxels(&p, p.domain_lo, p.domain_hi) == 7 * 7 * 7);

    MechParams bad = p;
    bad.voxel_size = 20.0;   /* smaller than 1.25 * 2 * 11 is fine for the workspace size */
    bad.abi_version = 0;
    CHECK(population_workspace_bytes(&bad, 10) == MECH_E_INVALID);
    CHECK(strlen(mech_last_error()) > 0);

    /* a cell outside the domain is rejected before any device call */
    double pos[3] = {0.0, 0.0, 150.0}, radius[1] = {8.4};
    MechPopulation* pop = (MechPopulation*)&p; /* must be reset to NULL on error */
    CHECK(create_population(&p, 1, pos, radius, NULL, NULL, NULL, &pop) == MECH_E_OUT_OF_DOMAIN);
    CHECK(pop == NULL);
    CHECK(step_mechanics(NULL, 1) == MECH_E_INVALID);
    CHECK(destroy_population(NULL) == MECH_OK);

    MechTuning t;
    CHECK(batch_get_tuning(NULL, &t) == MECH_E_INVALID);

    /* byte-budget arenas: capacity grows with the budget, none fits in 1 KiB */
    int64_t c1 = 0, v1 = 0, c2 = 0, v2 = 0;
    CHECK(batch_budget_capacity(&p, (int64_t)1 << 30, 1.6, 16, &c1, &v1) == MECH_OK);
    CHECK(batch_budget_capacity(&p, (int64_t)2 << 30, 1.6, 16, &c2, &v2) == MECH_OK);
    CHECK(c1 > 0 && c2 > c1 && v2 >= v1);
    CHECK(batch_budget_capacity(&p, 1024, 1.6, 16, &c1, &v1) == MECH_E_BUDGET);

    /* the allocation-free call validates on the host before touching a device */
    double out[3];
    CHECK(step_mechanics_noalloc(&bad, 1, pos, radius, NULL, NULL, 1, NULL, out, NULL, NULL) == MECH_E_INVALID);
    CHECK(step_mechanics_noalloc(&p, 1, pos, radius, NULL, NULL, 1, NULL, out, NULL, NULL) ==
          MECH_E_OUT_OF_DOMAIN);
    {
        const int64_t n = 400000;   /* more than the static scratch holds */
        double* big = malloc(sizeof(double) * 3 * (size_t)n);
        double* rad = malloc(sizeof(double) * (size_t)n);
        double* bout = malloc(sizeof(double) * 3 * (size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            for (int a = 0; a < 3; ++a) big[3 * i + a] = -90.0 + 180.0 * (double)((i * (a + 7)) % 1000) / 1000.0;
            rad[i] = 8.4;
        }
        CHECK(step_mechanics_noalloc(&p, n, big, rad, NULL, NULL, 1, NULL, bout, NULL, NULL) == MECH_E_NOMEM);
        free(big);
        free(rad);
        free(bout);
    }

    /* the microenvironment rejects bad parameters on the host */
    MechMicroenvParams mp;
    memset(&mp, 0, sizeof mp);
    mp.abi_version = MECH_ABI_VERSION;
    mp.n_substrates = 1;
    mp.dims[0] = mp.dims[1] = mp.dims[2] = 8;
    mp.voxel_size = 20.0;
    mp.dt = 0.01;
    mp.diffusion[0] = 1e5;
    mp.decay[0] = 0.1;
    MechMicroenv* env = (MechMicroenv*)&mp;
    mp.dims[1] = 0;
    CHECK(create_microenvironment(&mp, NULL, NULL, &env) == MECH_E_INVALID);
    CHECK(env == NULL);
    mp.dims[1] = 8;
    mp.decay[0] = -1.0;
    CHECK(create_microenvironment(&mp, NULL, NULL, &env) == MECH_E_INVALID);
    CHECK(microenvironment_step(NULL, 1) == MECH_E_INVALID);
    CHECK(destroy_microenvironment(NULL) == MECH_OK);
    printf("%s\n", fails ? "client failed" : "client ok");
    return fails ? 1 : 0;
}
