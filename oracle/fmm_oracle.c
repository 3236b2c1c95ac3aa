/*
 * fmm_oracle.c -- plain, slow, obviously-correct FP64 reference for the 2D
 * harmonic-kernel fast multipole method of Holm, Engblom, Goude & Holmgren,
 * "Dynamic autotuning of adaptive fast multipole methods on hybrid multicore
 * CPU & GPU systems" (arXiv:1311.1006).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * Contents
 *   O1  direct summation, eq. (2.1)/(2.2), exclusion by position, plus a
 *       Neumaier-compensated variant (reference of the reference);
 *   O2  serial FMM on the balanced ("pyramid") median-split tree of Sec. 2.2,
 *       with the strong / weak / decoupled connectivity of Sec. 2.1 and the
 *       theta-criterion (2.3), in the unscaled textbook form of the
 *       multipole / local expansions (Sec. 2.1, harmonic kernel of Sec. 3.3);
 *   O1s the same sum with the Gaussian smoother of Sec. 5.1 (eq. 5.2);
 *   O3  analytic gradient of a real loss through the direct sum, and the
 *       derivative of the field at separate evaluation points;
 *   the p(TOL, theta) rule that reproduces Table 4.1.
 *
 * Conventions
 *   Complex numbers are interleaved doubles (re, im).  The kernel is
 *   phi(z_i) = sum_{z_j != z_i} m_j / (z_i - z_j); the paper's harmonic
 *   potential -m_j/(x_i - x_j) (Sec. 3.3) differs by the global sign only.
 *   p is the number of expansion terms (k = 0..p-1).  Levels run 0..L-1 with
 *   the root at level 0 and N_f = 4^(L-1) leaves (Sec. 2.3).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 * The floating-point contract is off so that every product and sum in the
 * geometry and the theta-test is rounded on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

static inline cplx c_make(double re, double im) { cplx c; c.re = re; c.im = im; return c; }
static inline cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static inline cplx c_sub(cplx a, cplx b) { return c_make(a.re - b.re, a.im - b.im); }
static inline cplx c_mul(cplx a, cplx b) {
    return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
static inline cplx c_scale(cplx a, double s) { return c_make(a.re * s, a.im * s); }
/* 1/w = conj(w)/|w|^2 */
static inline cplx c_inv(cplx w) {
    double q = 1.0 / (w.re * w.re + w.im * w.im);
    return c_make(w.re * q, -w.im * q);
}
/* m / w for the kernel term; the caller guarantees w != 0 */
static inline cplx c_div(cplx m, cplx w) {
    double q = 1.0 / (w.re * w.re + w.im * w.im);
    return c_make((m.re * w.re + m.im * w.im) * q, (m.im * w.re - m.re * w.im) * q);
}

static inline cplx ld(const double* a, int64_t i) { return c_make(a[2 * i], a[2 * i + 1]); }
static inline void st(double* a, int64_t i, cplx v) { a[2 * i] = v.re; a[2 * i + 1] = v.im; }

/* ------------------------------------------------------------------------ */
/* O1: direct summation, eq. (2.1) and (2.2).  Sources with the same position
 * as the evaluation point are left out (the x_j != y_i of (2.2)); for
 * distinct points this is the j != i of (2.1).  Sum over j in input order.  */
/* ------------------------------------------------------------------------ */

/* Evaluate at the sources themselves (targets == NULL) or at the source
 * points listed in targets[0..nt). */
void oracle_direct(int64_t n, const double* z, const double* m, int64_t nt,
                   const int64_t* targets, double* phi)
{
    int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t i = targets ? targets[t] : t;
        cplx zi = ld(z, i), acc = c_make(0.0, 0.0);
        for (int64_t j = 0; j < n; ++j) {
            cplx w = c_sub(zi, ld(z, j));
            if (w.re == 0.0 && w.im == 0.0) continue;
            acc = c_add(acc, c_div(ld(m, j), w));
        }
        st(phi, t, acc);
    }
}

/* Evaluation at separate points y (eq. 2.2). */
void oracle_direct_points(int64_t n, const double* z, const double* m,
                          int64_t ny, const double* y, double* phi)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ny; ++t) {
        cplx yi = ld(y, t), acc = c_make(0.0, 0.0);
        for (int64_t j = 0; j < n; ++j) {
            cplx w = c_sub(yi, ld(z, j));
            if (w.re == 0.0 && w.im == 0.0) continue;
            acc = c_add(acc, c_div(ld(m, j), w));
        }
        st(phi, t, acc);
    }
}

/* Direct sum with the Gaussian smoother of the vortex application (Sec. 5.1,
 * eq. 5.2): every term m_j / (z_i - z_j) is multiplied by
 * g_delta(r) = 1 - exp(-r^2 / delta^2), r = |z_i - z_j|, which takes the
 * divergence out as z_j -> z_i; coincident positions are left out as above
 * (their smoothed term is 0).  Evaluated at the sources themselves
 * (targets == NULL) or at the listed ones. */
void oracle_direct_smoothed(int64_t n, const double* z, const double* m, double delta, int64_t nt,
                            const int64_t* targets, double* phi)
{
    int64_t cnt = targets ? nt : n;
    const double id2 = 1.0 / (delta * delta);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t i = targets ? targets[t] : t;
        cplx zi = ld(z, i), acc = c_make(0.0, 0.0);
        for (int64_t j = 0; j < n; ++j) {
            cplx w = c_sub(zi, ld(z, j));
            if (w.re == 0.0 && w.im == 0.0) continue;
            double r2 = w.re * w.re + w.im * w.im;
            double g = 1.0 - exp(-r2 * id2);
            acc = c_add(acc, c_scale(c_div(ld(m, j), w), g));
        }
        st(phi, t, acc);
    }
}

/* The logarithmic potential, the second kernel of the paper (end of Sec. 3;
 * the multipole expansion with its a_0 log term sits at the start of Sec. 2):
 * for real strengths q the real part of sum_j q_j log(y_i - z_j), i.e.
 *     u_i = sum over j with z_j != y_i of q_j log|y_i - z_j|,
 * single-valued (the imaginary part would depend on the branch of the
 * logarithm).  Sources at the evaluation point are left out, as in (2.1). */
void oracle_direct_log_points(int64_t n, const double* z, const double* q,
                              int64_t ny, const double* y, double* u)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ny; ++t) {
        cplx yi = ld(y, t);
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            cplx w = c_sub(yi, ld(z, j));
            if (w.re == 0.0 && w.im == 0.0) continue;
            acc += q[j] * log(hypot(w.re, w.im));
        }
        u[t] = acc;
    }
}

/* Derivative of the field of eq. (2.2) at separate points y: the y-derivative
 * of m_j / (y - x_j) is -m_j / (y - x_j)^2; sources at the evaluation point
 * are left out, as in the potential.  Evaluating at the sources themselves
 * (y = z) gives the derivative of (2.1)'s field with the self term removed. */
void oracle_direct_deriv_points(int64_t n, const double* z, const double* m,
                                int64_t ny, const double* y, double* dphi)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ny; ++t) {
        cplx yi = ld(y, t), acc = c_make(0.0, 0.0);
        for (int64_t j = 0; j < n; ++j) {
            cplx w = c_sub(yi, ld(z, j));
            if (w.re == 0.0 && w.im == 0.0) continue;
            cplx iw = c_inv(w);
            acc = c_sub(acc, c_mul(ld(m, j), c_mul(iw, iw)));
        }
        st(dphi, t, acc);
    }
}

/* Same sum with Neumaier (improved Kahan-Babuska) compensation of the real
 * and imaginary accumulators; used only at small N to check O1 itself. */
static inline void neumaier(double* s, double* c, double v) {
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v; else *c += (v - t) + *s;
    *s = t;
}

void oracle_direct_compensated(int64_t n, const double* z, const double* m, double* phi)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx zi = ld(z, i);
        double sr = 0, cr = 0, si = 0, ci = 0;
        for (int64_t j = 0; j < n; ++j) {
            cplx w = c_sub(zi, ld(z, j));
            if (w.re == 0.0 && w.im == 0.0) continue;
            cplx v = c_div(ld(m, j), w);
            neumaier(&sr, &cr, v.re);
            neumaier(&si, &ci, v.im);
        }
        st(phi, i, c_make(sr + cr, si + ci));
    }
}

/* ------------------------------------------------------------------------ */
/* O3: gradient of a real loss L(phi) through the direct sum.
 * Convention: for a complex quantity w, G_w = dL/dRe(w) + i dL/dIm(w).
 * Input g = G_phi.  With Phi[s](z_k) = sum_{i != k} s_i/(z_k - z_i),
 * psi_k = sum_{j != k} m_j/(z_k - z_j)^2 and chi_k = sum_{i != k} conj(g_i)/(z_k - z_i)^2,
 *   G_m_k = -conj(Phi[conj(g)](z_k)),
 *   G_z_k = -g_k conj(psi_k) + conj(m_k) conj(chi_k).
 * Derivation: phi is holomorphic in every m_j and z_j, so
 * dL = Re(sum_i conj(g_i) dphi_i); dphi_i/dm_k = 1/(z_i - z_k) for k != i,
 * dphi_i/dz_i = -psi_i, dphi_i/dz_k = m_k/(z_i - z_k)^2.                    */
/* ------------------------------------------------------------------------ */
void oracle_grad_direct(int64_t n, const double* z, const double* m, const double* g,
                        double* gm, double* gz)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        cplx zk = ld(z, k);
        cplx phi_g = c_make(0, 0), psi = c_make(0, 0), chi = c_make(0, 0);
        for (int64_t i = 0; i < n; ++i) {
            cplx w = c_sub(zk, ld(z, i));
            if (w.re == 0.0 && w.im == 0.0) continue;
            cplx iw = c_inv(w);
            cplx iw2 = c_mul(iw, iw);
            cplx gb = ld(g, i); gb.im = -gb.im;
            phi_g = c_add(phi_g, c_mul(gb, iw));
            psi = c_add(psi, c_mul(ld(m, i), iw2));
            chi = c_add(chi, c_mul(gb, iw2));
        }
        cplx gk = ld(g, k), mk = ld(m, k);
        st(gm, k, c_make(-phi_g.re, phi_g.im));                    /* -conj(Phi) */
        cplx psic = c_make(psi.re, -psi.im), chic = c_make(chi.re, -chi.im);
        cplx mkc = c_make(mk.re, -mk.im);
        cplx t1 = c_mul(gk, psic), t2 = c_mul(mkc, chic);
        st(gz, k, c_make(t2.re - t1.re, t2.im - t1.im));
    }
}

/* ------------------------------------------------------------------------ */
/* Expansion operators, unscaled textbook form for the harmonic kernel.
 * Outgoing (multipole) expansion about c of the sources in a box:
 *     phi(z) ~ sum_{k<p} a_k / (z - c)^(k+1),  a_k = sum_j m_j (z_j - c)^k,
 * from 1/(z - z_j) = sum_k (z_j - c)^k / (z - c)^(k+1).
 * Incoming (local) expansion about c:  phi(z) ~ sum_{l<p} b_l (z - c)^l.
 * Sec. 2.1 defines the two expansions and the shifts between them; the
 * formulas below are their form for the derivative (harmonic) kernel.       */
/* ------------------------------------------------------------------------ */

static double* binom_table(int nmax)
{
    double* C = (double*)calloc((size_t)(nmax + 1) * (nmax + 1), sizeof(double));
    for (int n = 0; n <= nmax; ++n) {
        C[n * (nmax + 1)] = 1.0;
        for (int k = 1; k <= n; ++k)
            C[n * (nmax + 1) + k] = C[(n - 1) * (nmax + 1) + k - 1] +
                                    (k <= n - 1 ? C[(n - 1) * (nmax + 1) + k] : 0.0);
    }
    return C;
}
#define BIN(C, nmax, n, k) ((C)[(n) * ((nmax) + 1) + (k)])

/* P2M: a_k += sum_j m_j (z_j - c)^k over the n given points. */
void oracle_p2m(const double* c, int64_t n, const double* z, const double* m, int p, double* a)
{
    cplx cc = c_make(c[0], c[1]);
    for (int64_t j = 0; j < n; ++j) {
        cplx w = c_sub(ld(z, j), cc), pw = c_make(1.0, 0.0), mj = ld(m, j);
        for (int k = 0; k < p; ++k) {
            st(a, k, c_add(ld(a, k), c_mul(mj, pw)));
            pw = c_mul(pw, w);
        }
    }
}

/* Evaluate a multipole expansion at n points: phi += sum_k a_k/(z - c)^(k+1).
 * Used by the tests to check P2M against its closed-form remainder. */
void oracle_mpole_eval(const double* c, int p, const double* a, int64_t n, const double* z, double* phi)
{
    cplx cc = c_make(c[0], c[1]);
    for (int64_t i = 0; i < n; ++i) {
        cplx iw = c_inv(c_sub(ld(z, i), cc)), pw = iw, acc = c_make(0, 0);
        for (int k = 0; k < p; ++k) {
            acc = c_add(acc, c_mul(ld(a, k), pw));
            pw = c_mul(pw, iw);
        }
        st(phi, i, c_add(ld(phi, i), acc));
    }
}

/* M2M: re-centre a child's multipole (about cc) to the parent centre cp and
 * add it:  a^P_k += sum_{l<=k} C(k,l) a^C_l (cc - cp)^(k-l).  Exact for the
 * retained terms, since a^P_k only involves a^C_l with l <= k. */
void oracle_m2m(const double* cc, const double* cp, int p, const double* ac, double* ap)
{
    double* C = binom_table(p);
    cplx d = c_make(cc[0] - cp[0], cc[1] - cp[1]);
    cplx* dp = (cplx*)malloc(sizeof(cplx) * (size_t)p);
    dp[0] = c_make(1, 0);
    for (int k = 1; k < p; ++k) dp[k] = c_mul(dp[k - 1], d);
    for (int k = 0; k < p; ++k) {
        cplx acc = c_make(0, 0);
        for (int l = 0; l <= k; ++l)
            acc = c_add(acc, c_scale(c_mul(ld(ac, l), dp[k - l]), BIN(C, p, k, l)));
        st(ap, k, c_add(ld(ap, k), acc));
    }
    free(dp); free(C);
}

/* M2L: multipole of source box S (about cs) into the local expansion of the
 * target box T (about ct), d = ct - cs:
 *   b_l += sum_k (-1)^l C(k+l, k) a_k / d^(k+l+1),
 * from 1/(d + w)^(k+1) = d^-(k+1) sum_l C(k+l, l) (-w/d)^l. */
void oracle_m2l(const double* cs, const double* ct, int p, const double* a, double* b)
{
    double* C = binom_table(2 * p);
    cplx d = c_make(ct[0] - cs[0], ct[1] - cs[1]);
    cplx id = c_inv(d);
    cplx* ip = (cplx*)malloc(sizeof(cplx) * (size_t)(2 * p + 1));
    ip[0] = c_make(1, 0);
    for (int k = 1; k <= 2 * p; ++k) ip[k] = c_mul(ip[k - 1], id);   /* d^-k */
    for (int l = 0; l < p; ++l) {
        cplx acc = c_make(0, 0);
        for (int k = 0; k < p; ++k)
            acc = c_add(acc, c_scale(c_mul(ld(a, k), ip[k + l + 1]), BIN(C, 2 * p, k + l, k)));
        if (l & 1) acc = c_scale(acc, -1.0);
        st(b, l, c_add(ld(b, l), acc));
    }
    free(ip); free(C);
}

/* L2L: re-centre a parent's local expansion (about cp) to a child centre cc
 * and add it:  b^C_l += sum_{k>=l} C(k,l) b^P_k (cc - cp)^(k-l).  Exact: it is
 * the same polynomial written about another point. */
void oracle_l2l(const double* cp, const double* cc, int p, const double* bp, double* bc)
{
    double* C = binom_table(p);
    cplx d = c_make(cc[0] - cp[0], cc[1] - cp[1]);
    cplx* dp = (cplx*)malloc(sizeof(cplx) * (size_t)p);
    dp[0] = c_make(1, 0);
    for (int k = 1; k < p; ++k) dp[k] = c_mul(dp[k - 1], d);
    for (int l = 0; l < p; ++l) {
        cplx acc = c_make(0, 0);
        for (int k = l; k < p; ++k)
            acc = c_add(acc, c_scale(c_mul(ld(bp, k), dp[k - l]), BIN(C, p, k, l)));
        st(bc, l, c_add(ld(bc, l), acc));
    }
    free(dp); free(C);
}

/* L2P: phi_i += sum_l b_l (z_i - c)^l. */
void oracle_l2p(const double* c, int p, const double* b, int64_t n, const double* z, double* phi)
{
    cplx cc = c_make(c[0], c[1]);
    for (int64_t i = 0; i < n; ++i) {
        cplx w = c_sub(ld(z, i), cc), pw = c_make(1, 0), acc = c_make(0, 0);
        for (int l = 0; l < p; ++l) {
            acc = c_add(acc, c_mul(ld(b, l), pw));
            pw = c_mul(pw, w);
        }
        st(phi, i, c_add(ld(phi, i), acc));
    }
}

/* ------------------------------------------------------------------------ */
/* Balanced ("pyramid") tree, Sec. 2.2.  Every leaf sits at level L-1 and the
 * boxes are split at the median so that leaf populations are (almost) equal.
 * The paper leaves the split rule to its source code; the reading used here:
 *   - a box is split into four by two successive binary splits;
 *   - each binary split cuts the longer side of the tight bounding box of the
 *     points being split (x when the sides are equal);
 *   - the points are ordered by (coordinate on that axis, input index) and the
 *     lower floor(n/2) of them form the first half;
 *   - children 4b+0, 4b+1 come from the first half, 4b+2, 4b+3 from the rest.
 * Box geometry: tight bounding box of the box's points, centre at its
 * midpoint and radius = half its diagonal (Sec. 2.1 speaks of box radii).
 * Requires 4^(L-1) <= n so that no box is empty.                            */
/* ------------------------------------------------------------------------ */

typedef struct { double x, y; int64_t idx; } opt;

static int cmp_x(const void* A, const void* B) {
    const opt* a = (const opt*)A; const opt* b = (const opt*)B;
    if (a->x < b->x) return -1;
    if (a->x > b->x) return 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}
static int cmp_y(const void* A, const void* B) {
    const opt* a = (const opt*)A; const opt* b = (const opt*)B;
    if (a->y < b->y) return -1;
    if (a->y > b->y) return 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

static void bbox_of(const opt* s, int64_t n, double* bb)
{
    double x0 = s[0].x, x1 = s[0].x, y0 = s[0].y, y1 = s[0].y;
    for (int64_t i = 1; i < n; ++i) {
        if (s[i].x < x0) x0 = s[i].x;
        if (s[i].x > x1) x1 = s[i].x;
        if (s[i].y < y0) y0 = s[i].y;
        if (s[i].y > y1) y1 = s[i].y;
    }
    bb[0] = x0; bb[1] = x1; bb[2] = y0; bb[3] = y1;
}

/* binary median split of s[0..n): returns the size of the lower half */
static int64_t halve(opt* s, int64_t n)
{
    double bb[4];
    bbox_of(s, n, bb);
    if (bb[1] - bb[0] >= bb[3] - bb[2]) qsort(s, (size_t)n, sizeof(opt), cmp_x);
    else                                qsort(s, (size_t)n, sizeof(opt), cmp_y);
    return n / 2;
}

/* Boxes of all levels are numbered level by level: box b of level l has the
 * flat index (4^l - 1)/3 + b.  Per box the tree stores
 *   range[2*f]   = first point (in tree order), range[2*f+1] = point count,
 *   geom[7*f..]  = xmin, xmax, ymin, ymax, cx, cy, r.
 * perm[t] = input index of the point at tree position t.                    */
int oracle_tree(int64_t n, const double* z, int L, int64_t* perm, int64_t* range, double* geom)
{
    if (L < 1 || n < 1) return -1;
    int64_t nleaf = (int64_t)1 << (2 * (L - 1));
    if (nleaf > n) return -1;
    opt* s = (opt*)malloc(sizeof(opt) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) { s[i].x = z[2 * i]; s[i].y = z[2 * i + 1]; s[i].idx = i; }
    range[0] = 0; range[1] = n;
    for (int l = 0; l + 1 < L; ++l) {
        int64_t nb = (int64_t)1 << (2 * l), base = (nb - 1) / 3, cbase = (4 * nb - 1) / 3;
        for (int64_t b = 0; b < nb; ++b) {
            int64_t s0 = range[2 * (base + b)], cnt = range[2 * (base + b) + 1];
            int64_t h = halve(s + s0, cnt);
            int64_t h0 = halve(s + s0, h);
            int64_t h1 = halve(s + s0 + h, cnt - h);
            int64_t* r = range + 2 * (cbase + 4 * b);
            r[0] = s0;          r[1] = h0;
            r[2] = s0 + h0;     r[3] = h - h0;
            r[4] = s0 + h;      r[5] = h1;
            r[6] = s0 + h + h1; r[7] = cnt - h - h1;
        }
    }
    int64_t nbox = ((int64_t)1 << (2 * L)) / 3;   /* (4^L - 1)/3 */
    for (int64_t f = 0; f < nbox; ++f) {
        double* g = geom + 7 * f;
        bbox_of(s + range[2 * f], range[2 * f + 1], g);
        g[4] = 0.5 * (g[0] + g[1]);
        g[5] = 0.5 * (g[2] + g[3]);
        double dx = g[1] - g[0], dy = g[3] - g[2];
        double dx2 = dx * dx, dy2 = dy * dy;
        g[6] = 0.5 * sqrt(dx2 + dy2);
    }
    for (int64_t t = 0; t < n; ++t) perm[t] = s[t].idx;
    free(s);
    return 0;
}

/* theta-criterion (2.3): boxes with radii r1, r2 and centre distance d are
 * well separated when R + theta*r <= theta*d, R = max, r = min.  Written
 * squared to avoid the square root; d > 0 is required, so a box is never
 * well separated from itself. */
int oracle_well_separated(const double* gb, const double* gc, double theta)
{
    double R = gb[6] > gc[6] ? gb[6] : gc[6];
    double rr = gb[6] > gc[6] ? gc[6] : gb[6];
    double dx = gb[4] - gc[4], dy = gb[5] - gc[5];
    double dx2 = dx * dx, dy2 = dy * dy;
    double s = dx2 + dy2;
    double tr = theta * rr;
    double t = R + tr;
    double tt = t * t;
    double th2 = theta * theta;
    double rhs = th2 * s;
    return (s > 0.0) && (tt <= rhs);
}

/* Connectivity, Sec. 2.1: a box is strongly coupled to itself; children of
 * strongly coupled boxes are strongly coupled unless they satisfy the
 * theta-criterion, in which case they are weakly coupled (interact by M2L at
 * that level); children of weakly coupled boxes are decoupled.  At the
 * finest level the strong pairs interact directly (P2P).
 * Lists are kept in ascending box order, CSR per level over level-local box
 * indices:  soff[lo .. lo + 4^l], sid[...], woff, wid, where lo = (4^l - 1)/3
 * + l is the offset of level l in the offset arrays.  The caller sizes the
 * id arrays from oracle_list_counts.                                         */
static int64_t lvl_base(int l) { return (((int64_t)1 << (2 * l)) - 1) / 3; }

/* counts of strong and weak entries per level (arrays of length L) */
void oracle_list_counts(int L, const double* geom, double theta, int64_t* nstrong, int64_t* nweak)
{
    /* strong lists of the previous level, as flat arrays */
    int64_t* poff = (int64_t*)malloc(sizeof(int64_t) * 2);
    int64_t* pid = (int64_t*)malloc(sizeof(int64_t));
    poff[0] = 0; poff[1] = 1; pid[0] = 0;
    nstrong[0] = 1; nweak[0] = 0;
    for (int l = 1; l < L; ++l) {
        int64_t nb = (int64_t)1 << (2 * l);
        const double* g = geom + 7 * lvl_base(l);
        int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb + 1));
        int64_t total = 0, wtotal = 0;
        for (int pass = 0; pass < 2; ++pass) {
            int64_t* ids = NULL;
            if (pass == 1) ids = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total ? total : 1));
            int64_t cur = 0;
            for (int64_t b = 0; b < nb; ++b) {
                if (pass == 0) off[b] = cur;
                int64_t P = b >> 2;
                for (int64_t e = poff[P]; e < poff[P + 1]; ++e)
                    for (int64_t c = 4 * pid[e]; c < 4 * pid[e] + 4; ++c) {
                        int ws = (c != b) && oracle_well_separated(g + 7 * b, g + 7 * c, theta);
                        if (ws) { if (pass == 0) ++wtotal; }
                        else { if (pass == 1) ids[cur] = c; ++cur; }
                    }
            }
            if (pass == 0) { off[nb] = cur; total = cur; }
            else { free(pid); pid = ids; }
        }
        free(poff); poff = off;
        nstrong[l] = total; nweak[l] = wtotal;
    }
    free(poff); free(pid);
}

/* fill the CSR lists of every level; offsets are per level with 4^l + 1
 * entries each, concatenated (level l starts at lvl_base(l) + l) */
void oracle_lists(int L, const double* geom, double theta,
                  int64_t* soff, int64_t* sid, int64_t* woff, int64_t* wid)
{
    soff[0] = 0; soff[1] = 1; sid[0] = 0;
    woff[0] = 0; woff[1] = 0;
    int64_t sbase = 1, wbase = 0;          /* start of level l's ids */
    int64_t psbase = 0;                    /* start of level l-1's ids */
    for (int l = 1; l < L; ++l) {
        int64_t nb = (int64_t)1 << (2 * l);
        int64_t ooff = lvl_base(l) + l, pooff = lvl_base(l - 1) + l - 1;
        const double* g = geom + 7 * lvl_base(l);
        int64_t sc = 0, wc = 0;
        for (int64_t b = 0; b < nb; ++b) {
            soff[ooff + b] = sc; woff[ooff + b] = wc;
            int64_t P = b >> 2;
            for (int64_t e = soff[pooff + P]; e < soff[pooff + P + 1]; ++e) {
                int64_t q = sid[psbase + e];
                for (int64_t c = 4 * q; c < 4 * q + 4; ++c) {
                    int ws = (c != b) && oracle_well_separated(g + 7 * b, g + 7 * c, theta);
                    if (ws) wid[wbase + wc++] = c;
                    else    sid[sbase + sc++] = c;
                }
            }
        }
        soff[ooff + nb] = sc; woff[ooff + nb] = wc;
        psbase = sbase;
        sbase += sc; wbase += wc;
    }
}

/* ------------------------------------------------------------------------ */
/* O2: the FMM itself, in the order of Sec. 2.1 (Fig. 2.2): P2M at the leaves,
 * M2M upward, then M2L at every level followed by L2L to the next level,
 * finally L2P at the leaves plus the direct P2P sum over the finest-level
 * strong lists.  phi_near / phi_far (optional) receive the two parts.       */
/* ------------------------------------------------------------------------ */
int oracle_fmm(int64_t n, const double* z, const double* m, int p, double theta, int L,
               double* phi, double* phi_near, double* phi_far)
{
    if (L < 1 || p < 1 || !(theta > 0.0 && theta < 1.0)) return -1;
    int64_t nleaf = (int64_t)1 << (2 * (L - 1));
    if (nleaf > n) return -1;
    int64_t nbox = ((int64_t)1 << (2 * L)) / 3;
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* range = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)nbox);
    double* geom = (double*)malloc(sizeof(double) * 7 * (size_t)nbox);
    if (oracle_tree(n, z, L, perm, range, geom)) return -1;

    int64_t* ns = (int64_t*)malloc(sizeof(int64_t) * (size_t)L);
    int64_t* nw = (int64_t*)malloc(sizeof(int64_t) * (size_t)L);
    oracle_list_counts(L, geom, theta, ns, nw);
    int64_t tot_s = 0, tot_w = 0;
    for (int l = 0; l < L; ++l) { tot_s += ns[l]; tot_w += nw[l]; }
    int64_t noff = nbox + L;
    int64_t* soff = (int64_t*)malloc(sizeof(int64_t) * (size_t)noff);
    int64_t* woff = (int64_t*)malloc(sizeof(int64_t) * (size_t)noff);
    int64_t* sid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(tot_s + 1));
    int64_t* wid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(tot_w + 1));
    oracle_lists(L, geom, theta, soff, sid, woff, wid);

    /* points and strengths in tree order */
    double* zt = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* mt = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    for (int64_t t = 0; t < n; ++t) {
        zt[2 * t] = z[2 * perm[t]]; zt[2 * t + 1] = z[2 * perm[t] + 1];
        mt[2 * t] = m[2 * perm[t]]; mt[2 * t + 1] = m[2 * perm[t] + 1];
    }
    double* A = (double*)calloc((size_t)nbox * 2 * (size_t)p, sizeof(double));  /* multipoles */
    double* B = (double*)calloc((size_t)nbox * 2 * (size_t)p, sizeof(double));  /* locals */
    double* far = (double*)calloc(2 * (size_t)n, sizeof(double));
    double* near = (double*)calloc(2 * (size_t)n, sizeof(double));
    int64_t lb = lvl_base(L - 1);

    /* P2M at the leaves */
    for (int64_t b = 0; b < nleaf; ++b) {
        int64_t f = lb + b;
        oracle_p2m(geom + 7 * f + 4, range[2 * f + 1], zt + 2 * range[2 * f], mt + 2 * range[2 * f],
                   p, A + 2 * p * f);
    }
    /* M2M upward: level l children into level l-1 parents, l = L-1 .. 2 */
    for (int l = L - 1; l >= 2; --l) {
        int64_t nb = (int64_t)1 << (2 * l);
        for (int64_t b = 0; b < nb; ++b) {
            int64_t f = lvl_base(l) + b, fp = lvl_base(l - 1) + (b >> 2);
            oracle_m2m(geom + 7 * f + 4, geom + 7 * fp + 4, p, A + 2 * p * f, A + 2 * p * fp);
        }
    }
    /* downward: M2L at level l, then L2L into level l+1 */
    int64_t wlev = 0;
    for (int l = 1; l < L; ++l) {
        int64_t nb = (int64_t)1 << (2 * l), ooff = lvl_base(l) + l;
        for (int64_t b = 0; b < nb; ++b) {
            int64_t f = lvl_base(l) + b;
            for (int64_t e = woff[ooff + b]; e < woff[ooff + b + 1]; ++e) {
                int64_t fs = lvl_base(l) + wid[wlev + e];
                oracle_m2l(geom + 7 * fs + 4, geom + 7 * f + 4, p, A + 2 * p * fs, B + 2 * p * f);
            }
        }
        wlev += woff[ooff + nb];
        if (l + 1 < L) {
            int64_t nc = (int64_t)1 << (2 * (l + 1));
            for (int64_t c = 0; c < nc; ++c) {
                int64_t fc = lvl_base(l + 1) + c, fp = lvl_base(l) + (c >> 2);
                oracle_l2l(geom + 7 * fp + 4, geom + 7 * fc + 4, p, B + 2 * p * fp, B + 2 * p * fc);
            }
        }
    }
    /* L2P at the leaves */
    for (int64_t b = 0; b < nleaf; ++b) {
        int64_t f = lb + b;
        oracle_l2p(geom + 7 * f + 4, p, B + 2 * p * f, range[2 * f + 1], zt + 2 * range[2 * f],
                   far + 2 * range[2 * f]);
    }
    /* P2P over the finest-level strong lists */
    {
        int64_t sl = 0;
        for (int l = 0; l + 1 < L; ++l) sl += ns[l];
        int64_t ooff = lb + (L - 1);
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = 0; b < nleaf; ++b) {
            int64_t f = lb + b;
            for (int64_t i = range[2 * f]; i < range[2 * f] + range[2 * f + 1]; ++i) {
                cplx zi = ld(zt, i), acc = c_make(0, 0);
                for (int64_t e = soff[ooff + b]; e < soff[ooff + b + 1]; ++e) {
                    int64_t fs = lb + sid[sl + e];
                    for (int64_t j = range[2 * fs]; j < range[2 * fs] + range[2 * fs + 1]; ++j) {
                        cplx w = c_sub(zi, ld(zt, j));
                        if (w.re == 0.0 && w.im == 0.0) continue;
                        acc = c_add(acc, c_div(ld(mt, j), w));
                    }
                }
                st(near, i, acc);
            }
        }
    }
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = perm[t];
        phi[2 * i] = far[2 * t] + near[2 * t];
        phi[2 * i + 1] = far[2 * t + 1] + near[2 * t + 1];
        if (phi_near) { phi_near[2 * i] = near[2 * t]; phi_near[2 * i + 1] = near[2 * t + 1]; }
        if (phi_far) { phi_far[2 * i] = far[2 * t]; phi_far[2 * i + 1] = far[2 * t + 1]; }
    }
    free(perm); free(range); free(geom); free(ns); free(nw); free(soff); free(woff);
    free(sid); free(wid); free(zt); free(mt); free(A); free(B); free(far); free(near);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Expansion order from tolerance.  Sec. 2.3 and Sec. 4 state p ~ log TOL /
 * log theta without the constant; the rule
 *     p = ceil( ln(kappa * TOL * (1 - theta)) / ln(theta) ),  kappa = 17,
 * reproduces all fifteen entries of Table 4.1 (any kappa in [16.5, 17.9]
 * does).  The (1 - theta) factor is the geometric-series tail of theta^k.   */
/* ------------------------------------------------------------------------ */
int oracle_p_from_tol(double tol, double theta)
{
    double v = log(17.0 * tol * (1.0 - theta)) / log(theta);
    return (int)ceil(v);
}

/* threads the OpenMP loops of this file use */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
