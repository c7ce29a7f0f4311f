/* A plain C client of libmech.so: builds against include/mech.h alone (no Python, no
 * torch types) and exercises the calls that need no GPU.  Run by test_abi.py. */
#include <stdio.h>
#include <string.h>

#include "mech.h"

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
    printf("%s\n", fails ? "client failed" : "client ok");
    return fails ? 1 : 0;
}
