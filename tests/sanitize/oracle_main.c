/*
 * oracle_main.c -- drives every entry of the CPU oracle once at small sizes
 * under AddressSanitizer and UndefinedBehaviorSanitizer (built by
 * tests/test_sanitize.py with the oracle's own source).  Exit status 0 when
 * every call returns and its return code is the expected one; the sanitizers
 * abort the process on any out-of-bounds access, leak or undefined operation.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_direct(int64_t, const double*, const double*, int64_t, const int64_t*, double*);
void oracle_direct_points(int64_t, const double*, const double*, int64_t, const double*, double*);
void oracle_direct_smoothed(int64_t, const double*, const double*, double, int64_t, const int64_t*, double*);
void oracle_direct_log_points(int64_t, const double*, const double*, int64_t, const double*, double*);
void oracle_direct_deriv_points(int64_t, const double*, const double*, int64_t, const double*, double*);
void oracle_direct_compensated(int64_t, const double*, const double*, double*);
void oracle_grad_direct(int64_t, const double*, const double*, const double*, double*, double*);
void oracle_p2m(const double*, int64_t, const double*, const double*, int, double*);
void oracle_mpole_eval(const double*, int, const double*, int64_t, const double*, double*);
void oracle_m2m(const double*, const double*, int, const double*, double*);
void oracle_m2l(const double*, const double*, int, const double*, double*);
void oracle_l2l(const double*, const double*, int, const double*, double*);
void oracle_l2p(const double*, int, const double*, int64_t, const double*, double*);
int oracle_tree(int64_t, const double*, int, int64_t*, int64_t*, double*);
int oracle_well_separated(const double*, const double*, double);
void oracle_list_counts(int, const double*, double, int64_t*, int64_t*);
void oracle_lists(int, const double*, double, int64_t*, int64_t*, int64_t*, int64_t*);
int oracle_fmm(int64_t, const double*, const double*, int, double, int, double*, double*, double*);
int oracle_p_from_tol(double, double);

static uint64_t state = 12345;
static double urand(void)   /* xorshift64*, uniform in [0, 1) */
{
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                   \
        }                                                              \
    } while (0)

static int64_t nbox(int L) { return (((int64_t)1 << (2 * L)) - 1) / 3; }

int main(void)
{
    const int64_t n = 700;
    double* z = malloc(sizeof(double) * 2 * n);
    double* m = malloc(sizeof(double) * 2 * n);
    double* out = malloc(sizeof(double) * 2 * n);
    double* out2 = malloc(sizeof(double) * 2 * n);
    double* near = malloc(sizeof(double) * 2 * n);
    double* far = malloc(sizeof(double) * 2 * n);
    double* g = malloc(sizeof(double) * 2 * n);
    double* q = malloc(sizeof(double) * n);
    int64_t* t = malloc(sizeof(int64_t) * 50);
    for (int64_t i = 0; i < n; ++i) {
        z[2 * i] = urand();
        z[2 * i + 1] = urand();
        m[2 * i] = urand() - 0.5;
        m[2 * i + 1] = urand() - 0.5;
        g[2 * i] = urand();
        g[2 * i + 1] = urand();
        q[i] = urand() - 0.5;
    }
    z[2 * 7] = z[2 * 3];            /* a coincident pair */
    z[2 * 7 + 1] = z[2 * 3 + 1];
    for (int i = 0; i < 50; ++i) t[i] = (i * 13) % n;

    oracle_direct(n, z, m, n, NULL, out);
    oracle_direct(n, z, m, 50, t, out2);
    CHECK(out2[0] == out[0] && out2[2 * 49] == out[2 * t[49]]);
    oracle_direct_points(n, z, m, 50, z, out2);
    oracle_direct_smoothed(n, z, m, 1e-3, 50, t, out2);
    oracle_direct_log_points(n, z, q, 50, z, out2);
    oracle_direct_deriv_points(n, z, m, 50, z, out2);
    oracle_direct_compensated(n, z, m, out2);
    oracle_grad_direct(n, z, m, g, out2, near);

    /* single operators at p = 1 and p = 64 */
    for (int p = 1; p <= 64; p += 63) {
        double c[2] = {0.5, 0.5}, c2[2] = {0.25, 0.25}, c3[2] = {3.0, 3.0};
        double* a = calloc(2 * (size_t)p, sizeof(double));
        double* b = calloc(2 * (size_t)p, sizeof(double));
        oracle_p2m(c, 20, z, m, p, a);
        oracle_mpole_eval(c, p, a, 5, z + 40, out2);
        oracle_m2m(c2, c, p, a, b);
        oracle_m2l(c, c3, p, a, b);
        oracle_l2l(c3, c2, p, b, a);
        oracle_l2p(c2, p, a, 5, z, out2);
        free(a);
        free(b);
    }

    /* tree, lists and the FMM at a few levels, an invalid level count */
    for (int L = 1; L <= 4; ++L) {
        const int64_t nb = nbox(L);
        int64_t* perm = malloc(sizeof(int64_t) * n);
        int64_t* range = malloc(sizeof(int64_t) * 2 * nb);
        double* geom = malloc(sizeof(double) * 7 * nb);
        CHECK(oracle_tree(n, z, L, perm, range, geom) == 0);
        CHECK(oracle_well_separated(geom, geom, 0.5) == 0);
        int64_t* ns = calloc(L, sizeof(int64_t));
        int64_t* nw = calloc(L, sizeof(int64_t));
        oracle_list_counts(L, geom, 0.5, ns, nw);
        int64_t ts = 0, tw = 0;
        for (int l = 0; l < L; ++l) { ts += ns[l]; tw += nw[l]; }
        int64_t* soff = calloc(nb + L, sizeof(int64_t));
        int64_t* woff = calloc(nb + L, sizeof(int64_t));
        int64_t* sid = calloc(ts + 1, sizeof(int64_t));
        int64_t* wid = calloc(tw + 1, sizeof(int64_t));
        oracle_lists(L, geom, 0.5, soff, sid, woff, wid);
        CHECK(oracle_fmm(n, z, m, 12, 0.5, L, out2, near, far) == 0);
        CHECK(oracle_fmm(n, z, m, 33, 0.65, L, out2, near, far) == 0);
        free(perm); free(range); free(geom); free(ns); free(nw); free(soff); free(woff); free(sid); free(wid);
    }
    {
        int64_t perm[16], range[2 * 21];
        double geom[7 * 21];
        CHECK(oracle_tree(16, z, 4, perm, range, geom) != 0);   /* 64 leaves > 16 points */
    }
    CHECK(oracle_p_from_tol(1e-6, 0.5) == 17);
    CHECK(oracle_p_from_tol(1e-8, 0.65) == 39);
    for (int64_t i = 0; i < 2 * n; ++i) CHECK(isfinite(out[i]));
    free(z); free(m); free(out); free(out2); free(near); free(far); free(g); free(q); free(t);
    if (fails) return 1;
    printf("oracle sanitizer run: ok\n");
    return 0;
}
