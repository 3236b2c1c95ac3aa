/*
 * host_main.c -- the host part of the C ABI (include/fmm.h) under
 * AddressSanitizer and UndefinedBehaviorSanitizer, without a GPU: argument
 * validation of every entry point (FMM_EINVAL, no handle created, a message
 * in fmm_last_error), the expansion-order rule of Table 4.1, and long runs
 * of the three autotuner walks on a synthetic clock.  Built and run by
 * tests/test_sanitize.py; exit status 0 when every check holds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/fmm.h"

static int fails = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                       \
        }                                                                  \
    } while (0)

static void expect_einval(int rc)
{
    CHECK(rc == FMM_EINVAL);
    CHECK(strlen(fmm_last_error()) > 0);
}

/* a time model with a minimum at n_levels = 7, theta = 0.5, split 2, batch 8 */
static double model(const fmm_tuner_params* p, int i)
{
    const double dl = p->n_levels - 7.0, dt = p->theta - 0.5;
    const double noise = 0.01 * ((i * 7919) % 13) / 13.0;
    return 1.0 + 0.2 * dl * dl + 4.0 * dt * dt + 0.05 * (p->p2p_split != 2) + 0.05 * (p->m2l_batch != 8) + noise;
}

int main(void)
{
    double z[8] = {0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8};
    int64_t off[3] = {0, 4, 4};
    int L[2] = {1, 1};
    fmm_tree_t tree = (fmm_tree_t)0x1;
    /* fmm_build_tree */
    expect_einval(fmm_build_tree(z, off, 0, L, NULL, &tree));
    CHECK(tree == NULL);
    expect_einval(fmm_build_tree(z, off, 2, L, NULL, &tree));   /* an empty problem */
    int64_t off1[2] = {0, 4};
    int Lbad[1] = {3};
    expect_einval(fmm_build_tree(z, off1, 1, Lbad, NULL, &tree));   /* 16 leaves > 4 points */
    Lbad[0] = 0;
    expect_einval(fmm_build_tree(z, off1, 1, Lbad, NULL, &tree));
    Lbad[0] = 17;
    expect_einval(fmm_build_tree(z, off1, 1, Lbad, NULL, &tree));
    expect_einval(fmm_build_tree(z, NULL, 1, L, NULL, &tree));
    expect_einval(fmm_build_tree(NULL, off1, 1, L, NULL, &tree));
    int64_t offneg[2] = {1, 4};
    expect_einval(fmm_build_tree(z, offneg, 1, L, NULL, &tree));
    expect_einval(fmm_build_tree(z, off1, 1, L, NULL, NULL));
    /* a valid call reaches the device part: an error, never a handle */
    fmm_tree_t t2 = (fmm_tree_t)0x1;
    CHECK(fmm_build_tree(z, off1, 1, L, NULL, &t2) != FMM_OK);
    CHECK(t2 == NULL);
    /* plans and evaluations on NULL handles */
    fmm_plan_t pl = (fmm_plan_t)0x1;
    expect_einval(fmm_plan(NULL, 10, 0.5, FMM_FP64, NULL, NULL, &pl));
    CHECK(pl == NULL);
    expect_einval(fmm_plan(NULL, 10, 0.5, FMM_FP64, NULL, NULL, NULL));
    expect_einval(fmm_evaluate(NULL, z, z, NULL));
    expect_einval(fmm_evaluate_parts(NULL, z, z, z, NULL));
    expect_einval(fmm_evaluate_field(NULL, z, z, z, NULL));
    expect_einval(fmm_evaluate_log(NULL, z, z, NULL));
    expect_einval(fmm_evaluate_adjoint(NULL, z, z, z, z, NULL));
    expect_einval(fmm_tree_update_positions(NULL, z, NULL));
    fmm_stats st;
    expect_einval(fmm_plan_stats(NULL, &st));
    int nl = 0;
    int64_t np = 0, nb = 0, ne = 0;
    expect_einval(fmm_tree_layout(NULL, 0, &nl, &np, &nb));
    expect_einval(fmm_tree_download(NULL, 0, NULL, NULL, NULL, NULL));
    expect_einval(fmm_plan_list_size(NULL, 0, 0, 0, &ne));
    expect_einval(fmm_plan_download_list(NULL, 0, 0, 0, NULL, NULL, NULL));
    int pout = 0;
    expect_einval(fmm_choose_order(NULL, z, 0.5, 1e-6, 8, 24, NULL, &pout, NULL));
    fmm_tree_destroy(NULL);
    fmm_plan_destroy(NULL);
    /* the order rule reproduces Table 4.1 */
    static const double tab[15][3] = {{1e-6, 0.35, 11}, {1e-6, 0.40, 13}, {1e-6, 0.50, 17}, {1e-6, 0.60, 24},
                                      {1e-6, 0.65, 28}, {1e-7, 0.35, 14}, {1e-7, 0.40, 16}, {1e-7, 0.50, 21},
                                      {1e-7, 0.60, 28}, {1e-7, 0.65, 34}, {1e-8, 0.35, 16}, {1e-8, 0.40, 18},
                                      {1e-8, 0.50, 24}, {1e-8, 0.60, 33}, {1e-8, 0.65, 39}};
    for (int i = 0; i < 15; ++i) CHECK(fmm_p_from_tol(tab[i][0], tab[i][1]) == (int)tab[i][2]);
    CHECK(fmm_p_from_tol(0.0, 0.5) == FMM_EINVAL);
    CHECK(fmm_p_from_tol(1e-6, 1.0) == FMM_EINVAL);
    /* the tuner: invalid configurations, then long walks of every algorithm */
    fmm_tuner_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    fmm_tuner_t tu = NULL;
    expect_einval(fmm_tuner_create(&cfg, &tu));
    CHECK(tu == NULL);
    expect_einval(fmm_tuner_create(NULL, &tu));
    for (int alg = 0; alg < 3; ++alg) {
        memset(&cfg, 0, sizeof(cfg));
        cfg.init.n_levels = 5;
        cfg.init.p2p_split = 4;
        cfg.init.m2l_batch = 4;
        cfg.init.p = 17;
        cfg.init.theta = 0.40;
        cfg.min_levels = 3;
        cfg.max_levels = 10;
        cfg.cap = 0.1;
        cfg.window = 2;
        cfg.knob_interval = 5;
        cfg.algorithm = alg;
        cfg.level_interval = 4;
        cfg.theta_interval = 3;
        cfg.fib_length = 4;
        cfg.theta_min = 0.30;
        cfg.theta_max = 0.70;
        cfg.theta_unit = 0.01;
        cfg.tol = 1e-6;
        cfg.seed = 99;
        CHECK(fmm_tuner_create(&cfg, &tu) == FMM_OK);
        for (int i = 0; i < 3000; ++i) {
            fmm_tuner_params p;
            CHECK(fmm_tuner_next(tu, &p) == FMM_OK);
            CHECK(p.n_levels >= 3 && p.n_levels <= 10);
            CHECK(p.theta >= 0.30 - 1e-12 && p.theta <= 0.70 + 1e-12);
            CHECK(p.p == fmm_p_from_tol(1e-6, p.theta));
            CHECK(fmm_tuner_observe(tu, model(&p, i)) == FMM_OK);
        }
        fmm_tuner_params best;
        double cost = -1, run = -1;
        CHECK(fmm_tuner_best(tu, &best, &cost, &run) == FMM_OK);
        CHECK(cost >= 0.0 && run > 0.0);
        if (alg != 2) CHECK(best.n_levels == 7);   /* the directed walks find the minimum */
        fmm_tuner_destroy(tu);
        tu = NULL;
    }
    expect_einval(fmm_tuner_next(NULL, NULL));
    if (fails) return 1;
    printf("host sanitizer run: ok\n");
    return 0;
}
