/*
 * fmm.h -- C ABI of the MI355X (gfx950) fast multipole library for the 2D
 * harmonic kernel
 *
 *     phi(z_i) = sum_{j : z_j != z_i} m_j / (z_i - z_j),
 *
 * following Holm, Engblom, Goude & Holmgren, "Dynamic autotuning of adaptive
 * fast multipole methods on hybrid multicore CPU & GPU systems"
 * (arXiv:1311.1006): eq. (2.1)/(2.2) for the sum, Sec. 2.1 for the
 * theta-criterion (2.3) and the strong / weak / decoupled connectivity, Sec.
 * 2.2 for the balanced ("pyramid") median-split tree, Sec. 2.3 for N_levels
 * and p, Sec. 3.3 for the harmonic potential (the paper writes it with the
 * opposite global sign).
 *
 * Conventions shared by every call
 *   - Complex arrays are interleaved doubles (re, im), i.e. 16 bytes per value.
 *   - Array arguments marked DEVICE are device pointers on the current HIP
 *     device; HOST arrays are ordinary host memory read during the call.
 *   - Every device-side effect is ordered on `stream` (a hipStream_t; NULL is
 *     the null stream).  Calls return once the work is enqueued unless noted.
 *   - Points of problem b are entries offsets[b] .. offsets[b+1]-1 of the
 *     caller's arrays ("input order"); outputs are in input order too.
 *   - Levels follow the paper: level 0 is the root, leaves are at level
 *     n_levels-1, and a problem has N_f = 4^(n_levels-1) leaves.
 *   - p is the number of expansion terms (coefficients k = 0 .. p-1).
 *   - Return value: FMM_OK (0) or a negative fmm_status; on error nothing is
 *     written to the outputs, no handle is created and no memory leaks.
 *     fmm_last_error() then returns a message (thread-local).  Errors of
 *     asynchronous device work surface as FMM_EDEVICE at a later call.
 *   - Handles are not thread-safe; use each from one host thread at a time.
 *     The library owns all tree and plan memory; the caller owns every array
 *     it passes in.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_tree_s* fmm_tree_t;
typedef struct fmm_plan_s* fmm_plan_t;

enum fmm_status {
    FMM_OK = 0,
    FMM_EINVAL = -1,   /* invalid argument (sizes, levels, p, theta, non-finite input) */
    FMM_ENOMEM = -2,   /* device or host allocation failed */
    FMM_EDEVICE = -3,  /* a HIP runtime call or an earlier kernel failed */
    FMM_ESTATE = -4    /* handle used in a state that does not allow the call */
};

enum fmm_precision {
    FMM_FP64 = 0,   /* every step in FP64 */
    FMM_MIXED = 1   /* P2P and M2L in FP32 (FP32 accumulation); FP64 box geometry,
                       theta-tests and position differences (P2P: z_i - z_j in FP64,
                       rounded once to FP32; M2L: the centre difference in FP64, then
                       1/d and the rescaling powers of r_S/d and -r_T/d in FP32);
                       expansions stored in FP32 */
};

/* Flags of fmm_tuning.flags */
enum {
    FMM_FLAG_GRAPH = 1,       /* capture fmm_evaluate's kernels in a hipGraph on first
                                 use and replay it on later calls with the same
                                 pointers and stream */
    FMM_FLAG_PHASE_TIMING = 2, /* record per-phase hipEvent timings into fmm_stats
                                 (adds one event pair per phase) */
    FMM_FLAG_LEVELWISE = 4    /* run the far field's upward and downward passes level
                                 by level (one launch per level of M2M and of L2L)
                                 instead of by subtrees (trees whose problems all
                                 have the same N_levels >= 3, p <= 32: P2M with two
                                 M2M levels, three-level M2M subtrees, and an L2P
                                 that shifts every ancestor's M2L sum into the
                                 leaves directly); the two agree up to rounding */
};

/* Launch-shape knobs of one plan; 0 means "choose automatically". */
typedef struct {
    int p2p_split;   /* P2P: lane subgroups per wavefront (1, 2, 4); each subgroup takes
                        its own targets and one source per lane */
    int m2l_batch;   /* M2L: pair slots of one box in each 16-pair MFMA block: 16 (one
                        box per wavefront), 8, 4, 2 or 1 (2, 4, 8 or 16 boxes share a
                        wavefront and its blocks; with 1 every MFMA column is one box);
                        automatic: 4 */
    int flags;       /* FMM_FLAG_* */
    int p2p_targets; /* P2P: targets per lane, 1, 2, 4, 8 or 16 (FP64: at most 8); a work item
                        then takes p2p_targets x (lane subgroups) targets of one leaf.  With
                        p2p_split 0 the subgroups are the most that shape allows (4: 1..4
                        targets per lane, 2: 8 or 16); a (targets, split) pair the kernel has
                        no shape for (4 subgroups with 8 or 16, 2 with 1, 1 with 1 or 2) is
                        FMM_EINVAL.  0: from the leaf size */
    double smooth_delta;   /* > 0: the near field (P2P) takes every term times the Gaussian
                              smoother g(r) = 1 - exp(-r^2/delta^2) of the vortex application
                              (Sec. 5.1, eq. 5.2); the far field is left unsmoothed, which is
                              exact to exp(-R^2/delta^2) with R the smallest leaf radius (the
                              points of two well-separated boxes are at least the larger
                              radius apart at theta <= 0.5), so delta should be well below the
                              leaf radii.  fmm_evaluate and fmm_evaluate_parts only. 0: none */
    int p2p_src_tile;      /* P2P: sources staged in LDS per pass of a work item, 64, 128 or
                              256, at most the LDS buffer (128 sources mixed, 192 FP64); a
                              list is summed in passes of this many sources.  0: the
                              buffer */
    int reserved;
} fmm_tuning;

/* Host-side statistics of a plan (list sizes for the work model and the
 * roofline, last measured phase times when FMM_FLAG_PHASE_TIMING is set). */
typedef struct {
    int64_t n_points;          /* total points over all problems */
    int64_t n_boxes;           /* boxes over all levels and problems */
    int64_t n_leaves;
    int64_t n_p2p_pairs;       /* sum over leaves of n_T * (sources in its strong list) */
    int64_t n_m2l_pairs;       /* weak-list entries over all levels */
    int64_t n_strong_entries;  /* finest-level strong-list entries */
    int p, precision, max_levels, nprob;
    double theta;
    /* microseconds of the phases of the last fmm_evaluate run with
       FMM_FLAG_PHASE_TIMING (0 otherwise), from events on its stream:
       upward = gather + P2M + M2M, m2l = the M2L kernel(s) alone,
       downward = L2P, p2p = near field, l2l (below) = the L2L sweep */
    double t_upward_us, t_m2l_us, t_downward_us, t_p2p_us, t_total_us;
    double t_tree_us, t_plan_us;   /* last fmm_build_tree / fmm_plan device time, if timed */
    double t_l2l_us;
    int64_t static_bytes;      /* working memory fmm_evaluate_static needs for this plan */
} fmm_stats;

/*
 * fmm_build_tree -- balanced median-split tree of Sec. 2.2 for nprob
 * independent problems.
 *   z        DEVICE, complex [offsets[nprob]]: source positions, input order.
 *   offsets  HOST, int64 [nprob+1], offsets[0] = 0, nondecreasing.
 *   nprob    >= 1.
 *   n_levels HOST, int [nprob]: levels per problem, 1 <= L <= 16 with
 *            4^(L-1) <= N_b (no empty box), N_b = offsets[b+1]-offsets[b] >= 1.
 *   stream   hipStream_t.
 *   out      receives the handle.
 * Split rule (the paper defers details to its code; the reading used here):
 * every box is split in four by two successive binary splits; each binary
 * split cuts the longer side of the tight bounding box of the points being
 * split (x when equal) and puts the floor(n/2) points smallest in
 * (coordinate, input index) in the first half.  Box geometry: tight bounding
 * box, centre at its midpoint, radius = half its diagonal.  The tree copies
 * the positions: z may be freed once the stream has passed this call.
 * The call does not wait for the device.  Non-finite positions are detected
 * on the device: fmm_tree_download on this tree, and the first call that
 * needs the lists of a plan on it (see fmm_plan), then return FMM_EINVAL
 * ("non-finite position").
 */
int fmm_build_tree(const double* z, const int64_t* offsets, int nprob, const int* n_levels,
                   void* stream, fmm_tree_t* out);

/*
 * fmm_tree_update_positions -- replace the positions of an existing tree
 * while keeping its geometry (box centres, radii, membership) frozen.
 *   z  DEVICE, complex [N], input order.
 * Plans built on the tree then evaluate the FMM of the new positions with
 * the old geometry: the operator whose exact derivative fmm_evaluate_adjoint
 * returns (used for finite-difference checks and small position updates).
 */
int fmm_tree_update_positions(fmm_tree_t t, const double* z, void* stream);

void fmm_tree_destroy(fmm_tree_t t);

/*
 * fmm_plan -- connectivity lists and launch structures for one (p, theta,
 * precision) on a tree (Sec. 2.1: self is strongly coupled; children of a
 * strong pair are strong unless the theta-criterion (2.3) R + theta r <=
 * theta d holds, then weak; children of weak pairs are decoupled; finest-level
 * strong pairs are summed directly).
 *   p          1 .. 64 expansion terms.
 *   theta      0 < theta < 1.
 *   precision  FMM_FP64 or FMM_MIXED.
 *   tune       HOST, optional (NULL = automatic).
 * The plan references the tree, which must outlive it.  The call does not
 * wait for the device: the list build is enqueued on `stream`, and the first
 * call that needs the lists (fmm_evaluate, fmm_evaluate_parts,
 * fmm_evaluate_adjoint, fmm_plan_stats, fmm_plan_list_size,
 * fmm_plan_download_list) reads its flags (one synchronisation of `stream`)
 * and, rarely, rebuilds the lists with larger pools.  An error found there
 * (non-finite positions in the tree: FMM_EINVAL) is returned by that call
 * and by every later call on the plan.
 */
int fmm_plan(fmm_tree_t t, int p, double theta, int precision, const fmm_tuning* tune,
             void* stream, fmm_plan_t* out);

void fmm_plan_destroy(fmm_plan_t pl);

/*
 * fmm_evaluate -- phi = FMM(m) (Sec. 2.1, Fig. 2.2: P2M, M2M, M2L, L2L, L2P,
 * P2P).
 *   m    DEVICE, complex [N] strengths, input order.
 *   phi  DEVICE, complex [N] output, input order (overwritten).
 * The plan keeps the local expansions of the last call for the adjoint.
 */
int fmm_evaluate(fmm_plan_t pl, const double* m, double* phi, void* stream);

/*
 * fmm_evaluate_static -- fmm_evaluate for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc).  Same operator, same kernels and the same results as
 * fmm_evaluate on the plan; the call itself allocates nothing.  The
 * evaluation's working memory (strengths in tree order, near-field source
 * records and sums, multipole and local coefficients, partial sums of split
 * lists) is taken from a fixed device array of the library, 64 MiB per GPU,
 * held from the first call on a GPU until the process ends.
 *   m    DEVICE, complex [N] strengths, input order.
 *   phi  DEVICE, complex [N] output, input order (overwritten).
 * The plan's lists must be final: evaluate it once with fmm_evaluate, or
 * call fmm_plan_stats, first (else FMM_ESTATE).  Must be called with the
 * tree's device current (else FMM_EINVAL).  A plan whose evaluation needs
 * more than 64 MiB (fmm_stats.static_bytes; about 75 B per point plus
 * 2 p x 8 B (mixed) or 2 p x 16 B (FP64) per box) is refused with
 * FMM_EINVAL.  The plan's own buffers and the state the adjoint reads are
 * left as they were.  All calls on one GPU share its array: calls that
 * overlap in time on one GPU (other streams, other threads) race.
 * Errors: FMM_EINVAL, FMM_ESTATE, FMM_EDEVICE.
 */
int fmm_evaluate_static(fmm_plan_t pl, const double* m, double* phi, void* stream);

/*
 * fmm_evaluate_parts -- same operator, near field (P2P) and far field
 * (expansions) returned separately; phi = near + far.  Either pointer may be
 * NULL.  For diagnostics and parity tests.
 */
int fmm_evaluate_parts(fmm_plan_t pl, const double* m, double* phi_near, double* phi_far,
                       void* stream);

/*
 * fmm_evaluate_field -- phi as fmm_evaluate, plus the derivative of the field
 * at every point,
 *     dphi_i = dphi/dz (z_i) = -sum_{z_j != z_i} m_j / (z_i - z_j)^2
 * (the y-derivative of eq. 2.2's field; in a vortex method the derivative of
 * the velocity, Sec. 5.1).  The near field is summed directly over the strong
 * lists, the far field is the derivative of each leaf's local expansion (Sec.
 * 2.1), whose truncation error is larger than that of phi by roughly the
 * factor p.  Evaluation points apart from the sources: fmm_evaluate_points.
 * phi, dphi: device complex128 [N], input order.  Errors as for
 * fmm_evaluate.
 */
int fmm_evaluate_field(fmm_plan_t pl, const double* m, double* phi, double* dphi, void* stream);

/*
 * fmm_evaluate_points -- the field of the sources at M evaluation points
 * apart from them (eq. 2.2),
 *     phi_y[i] = sum_{x_j != y_i} m_j / (y_i - x_j),
 * and, when dphi_y is not NULL, its derivative
 *     dphi_y[i] = -sum_{x_j != y_i} m_j / (y_i - x_j)^2.
 * The plan is one over the sources' tree (Sec. 2.2) and lists (Sec. 2.1):
 * the points join neither, so they change no box and no list of the
 * sources.  Each point goes down the tree into the deepest box B whose
 * bounding box holds it; B's complete local expansion gives the field of the
 * sources outside B's strong list (it converges there: the point lies in the
 * boxes the theta-criterion was applied to), and each box of that list is
 * descended: a box well separated from the point (criterion (2.3) for a box
 * of radius zero) adds its multipole expansion at the point, a leaf that is
 * not adds its sources directly, other boxes are opened.  A point outside
 * the root's box is handled from the root down.  Accuracy as for
 * fmm_evaluate at the plan's p and theta.
 *   pl      a plan over a tree of ONE problem (else FMM_EINVAL) without a
 *           smoothed near field (else FMM_EINVAL);
 *   m       DEVICE, complex [N] source strengths, input order;
 *   y       DEVICE, complex [M] evaluation points;
 *   phi_y   DEVICE, complex [M] output;
 *   dphi_y  DEVICE, complex [M] output, or NULL for none;
 *   M       0 <= M < 2^31 - 1; M = 0: nothing is done.
 * A point that is not finite receives NaN.  The call allocates device
 * memory for the point order (8 B per point and 12 B per box), and leaves
 * the far field of m in the plan's buffers, not a forward evaluation:
 * fmm_evaluate_adjoint then needs a new fmm_evaluate first.  Errors:
 * FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE.
 */
int fmm_evaluate_points(fmm_plan_t pl, const double* m, const double* y, int64_t M, double* phi_y, double* dphi_y,
                        void* stream);

/*
 * fmm_evaluate_log -- the logarithmic potential, the second kernel of the
 * paper (Sec. 3.3), for real strengths:
 *     u_i = sum_{z_j != z_i} q_j log|z_i - z_j|
 * (the real part of sum_j q_j log(z_i - z_j); the imaginary part depends on
 * the branch of the logarithm and is not formed).  The far field uses the
 * multipole expansion a_0 log(z - z0) + sum_k a_k / (z - z0)^k of Sec. 2.1:
 * the harmonic expansions of the plan (the derivative of the potential) plus
 * a constant term per box, formed by M2L over the weak list and handed down
 * by L2L; the near field is summed directly over the strong lists.
 *   q  DEVICE, real float64 [N] strengths, input order.
 *   u  DEVICE, real float64 [N] output, input order (overwritten).
 * Separate evaluation points: as for fmm_evaluate_field, with zero strength.
 * Errors as for fmm_evaluate; FMM_EINVAL for a plan with a smoothed near
 * field.  Runs eagerly on `stream` also for a plan with FMM_FLAG_GRAPH; the
 * plan's state for fmm_evaluate_adjoint is cleared.
 */
int fmm_evaluate_log(fmm_plan_t pl, const double* q, double* u, void* stream);

/*
 * fmm_evaluate_adjoint -- gradients of a real loss L through phi = FMM(m; z)
 * with the tree geometry frozen.  Convention: for a complex w,
 * G_w = dL/dRe(w) + i dL/dIm(w).
 *   m      DEVICE, complex [N], the strengths of the forward call.
 *   g_phi  DEVICE, complex [N], G_phi (input order).
 *   g_m    DEVICE, complex [N], output G_m (may be NULL).
 *   g_z    DEVICE, complex [N], output G_z (may be NULL).
 * Runs the transposed chain (P2P^T, L2P^T, L2L^T, M2L^T, M2M^T, P2M^T) plus
 * the position derivatives of P2P, P2M and L2P.  Needs a preceding
 * fmm_evaluate with the same m on this plan (it reuses its local expansions).
 */
int fmm_evaluate_adjoint(fmm_plan_t pl, const double* m, const double* g_phi,
                         double* g_m, double* g_z, void* stream);

/* Fill *st (HOST).  Does not synchronise. */
int fmm_plan_stats(fmm_plan_t pl, fmm_stats* st);

/* ---- inspection (copies to HOST, synchronise `stream`) ------------------ */

/*
 * fmm_tree_layout -- sizes of problem `prob`: *n_levels, *n_points and the
 * number of boxes over all levels ((4^L - 1)/3).
 */
int fmm_tree_layout(fmm_tree_t t, int prob, int* n_levels, int64_t* n_points, int64_t* n_boxes);

/*
 * fmm_tree_download -- tree of problem `prob`, boxes numbered level by level
 * (box b of level l has index (4^l-1)/3 + b):
 *   perm   int64 [N_b]: input index (within the problem) of tree position t.
 *   range  int64 [n_boxes][2]: first tree position and point count per box.
 *   geom   double [n_boxes][7]: xmin, xmax, ymin, ymax, cx, cy, r.
 * Any pointer may be NULL.
 */
int fmm_tree_download(fmm_tree_t t, int prob, int64_t* perm, int64_t* range, double* geom,
                      void* stream);

/*
 * fmm_plan_list_size / fmm_plan_download_list -- connectivity of problem
 * `prob` at `level`, kind 0 = strong, 1 = weak, CSR over level-local box
 * indices: off int64 [4^level + 1], ids int64 [*n_entries], ascending per box.
 */
int fmm_plan_list_size(fmm_plan_t pl, int prob, int level, int kind, int64_t* n_entries);
int fmm_plan_download_list(fmm_plan_t pl, int prob, int level, int kind, int64_t* off,
                           int64_t* ids, void* stream);

/* ---- autotuner (host only) ---------------------------------------------- */

/*
 * Online autotuner after Sec. 4.2, fed one measured iteration time per call.
 * Rules kept from Sec. 4.2: a move is accepted or rejected on the timings
 * that follow it; noise is handled by judging a configuration by the minimum
 * time over a short window (window = 1 compares single iterations, as the
 * algorithms are printed); N_levels moves first when due, then theta, then
 * the launch-shape knobs.  Three walks (`algorithm`):
 *   FMM_TUNER_AT3B (Algorithm 4): directed walk; after a rejected N_levels
 *     move the next move in that direction is scheduled so that the
 *     accumulated cost of rejected moves stays below `cap` times the run
 *     time; theta moves as in AT2; in addition the P2P split and M2L batch
 *     knobs walk every knob_interval iterations, reversing on rejection.
 *   FMM_TUNER_AT2 (Algorithm 2): directed walk; N_levels moves every
 *     level_interval iterations in its current direction, reversed on
 *     rejection; theta moves every theta_interval iterations by
 *     thetastep * theta_unit in its direction; a rejected theta move reverses
 *     the direction and takes the next step length of a Fibonacci cycle
 *     (fib(1), fib(2), ... up to fib(fiblength - 1), then back to fib(1) with
 *     fiblength one longer), so that a walk held at an apparent optimum probes
 *     ever farther on both sides.
 *   FMM_TUNER_AT1 (Algorithm 1): random walk; N_levels (every level_interval
 *     iterations) and theta (every theta_interval, one theta_unit) move in a
 *     random direction (a SplitMix64 stream from `seed`).
 * theta stays on the grid theta_min + k * theta_unit inside
 * [theta_min, theta_max]; a move that would leave it is turned back (AT2,
 * AT3b) or mirrored (AT1).  theta_interval = 0 keeps theta at init.theta.
 * With tol > 0 every parameter set carries p = fmm_p_from_tol(tol, theta)
 * (Table 4.1's rule), so that theta acts as a pure performance knob (Sec.
 * 2.3); with tol = 0 p stays at init.p.
 */
typedef struct fmm_tuner_s* fmm_tuner_t;

enum { FMM_TUNER_AT3B = 0, FMM_TUNER_AT2 = 1, FMM_TUNER_AT1 = 2 };

typedef struct {
    int n_levels;
    int p2p_split;              /* walked over 1, 2, 4 (AT3b) */
    int m2l_batch;              /* walked over 1, 2, 4, 8, 16 (AT3b) */
    int p;                      /* expansion order for theta (see tol) */
    double theta;
} fmm_tuner_params;

typedef struct {
    fmm_tuner_params init;      /* starting point */
    int min_levels, max_levels; /* N_levels range (inclusive) */
    double cap;                 /* max tuning cost / run time, e.g. 0.1 (AT3b) */
    int window;                 /* iterations whose minimum time decides a move (>= 1) */
    int knob_interval;          /* iterations between P2P/M2L knob moves (>= 1, AT3b) */
    int algorithm;              /* FMM_TUNER_AT3B, FMM_TUNER_AT2 or FMM_TUNER_AT1 */
    int level_interval;         /* iterations between N_levels moves (AT1, AT2; >= 1) */
    int theta_interval;         /* iterations between theta moves; 0: theta fixed */
    int fib_length;             /* initial Fibonacci cycle length (>= 2; AT2, AT3b) */
    double theta_min, theta_max, theta_unit;   /* theta grid, e.g. 0.3, 0.7, 0.01 */
    double tol;                 /* > 0: p from tol and theta; 0: p fixed */
    unsigned long long seed;    /* AT1 directions */
} fmm_tuner_config;

int fmm_tuner_create(const fmm_tuner_config* cfg, fmm_tuner_t* out);
/* parameters to use for the next FMM call */
int fmm_tuner_next(fmm_tuner_t tu, fmm_tuner_params* out);
/* report the measured time (seconds) of the call made with the last parameters */
int fmm_tuner_observe(fmm_tuner_t tu, double seconds);
/* current best parameters and the tuning cost spent so far */
int fmm_tuner_best(fmm_tuner_t tu, fmm_tuner_params* best, double* cost_s, double* run_s);
void fmm_tuner_destroy(fmm_tuner_t tu);

/* Expansion order from tolerance: smallest p with the rule
 * p = ceil(ln(17 TOL (1-theta)) / ln theta), which reproduces Table 4.1. */
int fmm_p_from_tol(double tol, double theta);

/*
 * fmm_choose_order -- expansion order from a measured error.  The rule above
 * bounds the worst case; the error actually reached on a point set is often
 * several orders of p smaller, since the truncation error falls
 * geometrically in p at fixed theta (Sec. 2.3).  This call measures it:
 * the reference is the FP64 evaluation of the same tree and strengths at
 * p_ref = 32 when p_hi <= 24, else at p_ref = min(64, p_hi + 16) (at
 * theta <= 0.5 the truncation error of p = 32 is below 1e-12 relative);
 * for p = p_lo .. p_hi the FP64 and the mixed-precision evaluations are
 * compared with it in the relative 2-norm over all targets,
 *     e(p) = ||phi_p - phi_ref||_2 / ||phi_ref||_2,
 * and *p_out receives the smallest p at which both are <= tol, or -1 when no
 * p in the range reaches it.  err_out (may be NULL) receives
 * [e_fp64(p), e_mixed(p)] at that p (at p_hi when none qualifies).
 *   t: tree (one problem or several; the norm runs over all points);
 *   m: device complex128 [N] strengths, as for fmm_evaluate;
 *   1 <= p_lo <= p_hi <= 48, 0 < theta < 1, 0 < tol < 1.
 * Device work on `stream`, temporary device memory of 2 N complex values
 * plus the plans' own; the call waits for the device.  Errors: FMM_EINVAL
 * (arguments, non-finite tree), FMM_ENOMEM, FMM_EDEVICE.
 */
int fmm_choose_order(fmm_tree_t t, const double* m, double theta, double tol, int p_lo, int p_hi,
                     void* stream, int* p_out, double* err_out);

/* Thread-local message of the last failing call ("" if none). */
const char* fmm_last_error(void);

/* Test hooks for the allocation-failure paths (no paper passage: they check
 * the error contract above).  fmm_debug_fail_alloc(after): the device
 * allocation that comes `after` allocations from now (0: the next one)
 * fails once with FMM_ENOMEM, as if the device were out of memory, in
 * whatever call makes it; after < 0 cancels a pending failure.  The
 * setting is process-wide (all devices and threads).  Always FMM_OK.
 * fmm_debug_live_blocks(&n): n = device blocks currently held by trees,
 * plans, schedules and evaluations; blocks the library keeps cached for
 * reuse are not counted, so a sequence of calls whose handles are all
 * destroyed returns n to its value before the sequence (schedules and
 * launch tables cached per tree layout aside).  FMM_EINVAL if live is
 * NULL. */
int fmm_debug_fail_alloc(int64_t after);
int fmm_debug_live_blocks(int64_t* live);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H */
