/*
 * cil.h -- C ABI of the MI355X (gfx950) implementation of the Correlation
 * Integral Likelihood hot path (Kazarnikov, Scheichl, Haario,
 * Marciniak-Czochra, arXiv 2203.14742).
 *
 * The hot path: many reaction-diffusion solves run from randomised initial
 * states to stationary patterns (Sec. 4.1, App. B.1.1), then the correlation
 * integral statistic over pattern sets (Sec. 2.1 eqs. eCDF and CIL), its
 * bootstrap resampling (Alg. 2bst, Alg. 3bst) and the Gaussian synthetic
 * likelihood (eqs. cil:CF and cil:CF_synth).
 *
 * Conventions for every entry point:
 *   - Return value: CIL_OK (0) or a negative CIL_E* code; no exceptions cross
 *     the ABI.  cil_last_error() gives a thread-local message for the last
 *     failing call on the calling thread.
 *   - "device" pointers are HIP device memory of the current device
 *     (hipGetDevice at call time), owned by the caller; the library never
 *     frees or reallocates them.  "host" pointers are ordinary host memory.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  Work is
 *     stream-ordered on it.  A call that returns results in host memory
 *     synchronises that stream before it returns; a call whose outputs are
 *     all device memory returns without synchronising.
 *   - The library keeps internal device workspaces, DCT tables, auxiliary
 *     streams, a pool of the device buffers simulate calls used (reused by
 *     later calls) and tuning state per device; cil_shutdown() frees them.  A
 *     simulate call with several grid sides runs each side's persistent
 *     kernel on an auxiliary stream forked from, and joined back into, the
 *     caller's stream.
 *   - Pattern layout (Sec. 2.1 "patterns s in R^d", App. B.1.1 grid values):
 *     one pattern is [species v: n x n row-major][species w: n x n row-major],
 *     d = 2 n^2; a pattern set is nA rows of d contiguous elements.
 */
#ifndef CIL_H
#define CIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    CIL_OK = 0,
    CIL_EINVAL = -1,        /* bad argument (message in cil_last_error)        */
    CIL_EUNSUPPORTED = -2,  /* valid but not supported by this library         */
    CIL_ENOMEM = -3,        /* device workspace allocation failed              */
    CIL_EDEVICE = -4,       /* HIP runtime error, or no gfx950 device          */
    CIL_ENOTSPD = -5,       /* covariance not positive definite                */
    CIL_ENONFINITE = -6     /* a solve produced a non-finite value             */
};
const char *cil_strerror(int status);
const char *cil_last_error(void);

/* ---------------------------------------------------------------- models */
/* Reaction-diffusion kinetics of Sec. 4.1 (eq. rdgen:
 * v_t = nu1 Lap v + f(v,w), w_t = nu2 Lap w + g(v,w)); parameter vector p:
 *   CIL_FHN          p = {mu, eps, alpha}: f = eps (w - alpha v), g = -v + mu w - w^3
 *   CIL_GM           p = {mu_v, mu_w}:     f = -mu_v v + v^2/w,  g = -mu_w w + v^2
 *   CIL_GM_SOURCE    p = {a, b}:           f = a - b v + v^2/w,  g = v^2 - w
 *                    (Gierer-Meinhardt with a source term; nu = {1, d})
 *   CIL_BRUSSELATOR  p = {A, B}:           f = A - (B+1) v + v^2 w, g = B v - v^2 w
 *   CIL_HEAT         no kinetics (f = g = 0); pure diffusion, for testing     */
typedef enum {
    CIL_FHN = 0,
    CIL_GM = 1,
    CIL_GM_SOURCE = 2,
    CIL_BRUSSELATOR = 3,
    CIL_HEAT = 4
} cil_model;

typedef enum {
    CIL_FP64 = 0,   /* state / patterns are double                           */
    CIL_FP32 = 1    /* state / patterns are float                            */
} cil_precision;

/* One solve: grid side n (n x n nodes, h = L/(n-1), App. B.1.1), domain
 * length L, diffusion coefficients nu = {nu1, nu2}, kinetic parameters p. */
typedef struct {
    int32_t n;
    int32_t reserved;
    double L;
    double nu[2];
    double p[4];
} cil_problem;

typedef enum {
    CIL_PATH_AUTO = 0,        /* fused LDS-resident stepper where supported, else plain */
    CIL_PATH_PLAIN = 1,       /* one kernel per stage, host-driven step loop           */
    CIL_PATH_FUSED = 2,       /* fused stepper (default variant); CIL_EUNSUPPORTED
                                 where not available (n not in {32, 64, 128}; FP64 n = 128) */
    CIL_PATH_FUSED_LINE = 3,  /* fused, one lane transforms a whole grid line        */
    CIL_PATH_FUSED_QUAD = 4   /* fused, a quad of lanes transforms a grid line       */
} cil_path;

/* Time stepping: IMEX Euler with step dt.  tol <= 0: exactly max_steps steps.
 * tol > 0: a solve stops at the first step s with s % check_every == 0 whose
 * residual max|u^s - u^{s-1}|/dt (both species, all nodes, evaluated in
 * FP64) is < tol, or at max_steps.  FP32 only: when the residual falls below
 * the FP32 floor fp32_floor_ulps * 2^-24 * max|u| / dt (the state can no
 * longer resolve the residual) and tol is below that floor, polish != 0
 * continues the solve on the GPU until tol is met, the result rounded back to
 * FP32 (on the fused quad-lane path at n = 32 and 64 inside the same
 * persistent launch, see CIL_OPT_POLISH_SEPARATE):
 *   CIL_POLISH_FP64 (1): FP64 steps;
 *   CIL_POLISH_REFINE (2): the same steps in the refinement form u = U + v,
 *     U held in FP64, the correction v stepped with the FP32 transforms
 *     against the FP64 residual of U (five-point stencil) and the exact
 *     change of the reaction terms, so FP32 rounding scales with the size of
 *     v and the iteration has no FP32 floor; U absorbs v every 200 steps or
 *     so.  On the fused quad-lane path at n = 32 and 64 (default shapes);
 *     elsewhere as CIL_POLISH_FP64.  The stop rule and its FP64 residual are
 *     those above.
 * polish == 0 stops the solve at its floor with status CIL_SOLVE_FP32_FLOOR.
 * Other values: CIL_EINVAL. */
typedef enum { CIL_POLISH_OFF = 0, CIL_POLISH_FP64 = 1, CIL_POLISH_REFINE = 2 } cil_polish;
typedef struct {
    double dt;
    int64_t max_steps;
    double tol;
    int32_t check_every;      /* >= 1 */
    int32_t path;             /* cil_path */
    int32_t polish;           /* cil_polish, FP32 only, see above */
    int32_t fp32_floor_ulps;  /* <= 0 selects the default 8 */
} cil_stepping;

typedef enum {
    CIL_SOLVE_OK = 0,
    CIL_SOLVE_NONFINITE = 1,   /* non-finite value seen at a residual evaluation */
    CIL_SOLVE_MAXSTEPS = 2,    /* tol > 0 not met within max_steps               */
    CIL_SOLVE_FP32_FLOOR = 3   /* FP32 stopped at its floor (polish == 0)        */
} cil_solve_status;

typedef struct {
    int64_t steps_taken;   /* steps applied to this solve                     */
    int64_t steps_fp64;    /* of which in the polish (FP32 calls)             */
    double final_resid;    /* residual of the last evaluated step (NaN if non-finite) */
    int32_t status;        /* cil_solve_status                                */
    int32_t reserved;
} cil_solve_report;

/* Homogeneous steady state (v0, w0) with f = g = 0 (Sec. 4.1): FHN (0,0);
 * GM (mu_w/mu_v, mu_w/mu_v^2); GM_SOURCE ((a+1)/b, ((a+1)/b)^2);
 * Brusselator (A, B/A); HEAT (0,0).  Host only. */
int cil_homogeneous_state(cil_model model, const double *p /*host[4]*/, double *v0w0 /*host[2]*/);

/* Run B independent solves in place (App. B.1.1 method-of-lines system,
 * integrated by IMEX Euler: explicit pointwise reaction from the old step,
 * implicit diffusion (I - dt nu Lap_h) solved exactly in the cosine basis
 * that diagonalises the ghost-copy Neumann Laplacian).
 *   probs        host[B]; grid sides may differ between solves.
 *   state        device; element type by prec; solve b occupies 2 n_b^2
 *                elements at element offset elem_offsets[b]; in: initial
 *                states, out: states after the last step taken.
 *   elem_offsets host[B] or NULL (then solves are packed back to back).
 *   reports      host[B] or NULL.
 * Returns CIL_ENONFINITE if any solve ended with status NONFINITE (the other
 * solves are still completed), CIL_EINVAL for n < 2, dt <= 0, max_steps < 0,
 * check_every < 1, unknown model, NULL state. */
int cil_simulate_patterns(cil_model model, cil_precision prec, const cil_problem *probs, int32_t B,
                          void *state, const int64_t *elem_offsets, const cil_stepping *stepping,
                          cil_solve_report *reports, void *hip_stream);

/* The same solves with a second-order IMEX stepper (semi-implicit BDF2; the
 * paper's integrators, Sec. 5.1 and App. B.2, are first order in time or
 * explicit).  Step 1 of every call is the IMEX-Euler step above; step s >= 2:
 *   r_s = (4 u^{s-1} - u^{s-2}) / 3 + (2 dt / 3) (2 F(u^{s-1}) - F(u^{s-2}))
 *   u^s = (I - (2 dt / 3) nu_s Lap_h)^{-1} r_s    (cosine-basis solve)
 * Its fixed points are the stationary solutions nu Lap_h u + F(u) = 0, as
 * for IMEX Euler.  Residual, stop rule, reports and errors as for
 * cil_simulate_patterns.  The history (u^{s-2}, F(u^{s-2})) lives for one
 * call only: a call that continues from a state the previous one left starts
 * again with an Euler step, so it is not the same as one uninterrupted run.
 * Back-ends: a fused persistent kernel (one workgroup per solve, one lane
 * per grid line, state and history resident in LDS) for n = 32 and, in FP32,
 * n = 64; the plain back-end (history in two state-sized device buffers from
 * the library's buffer pool) otherwise.  Path AUTO picks the fused kernel
 * where it exists, PLAIN forces the plain back-end, FUSED and FUSED_LINE
 * require the fused kernel (CIL_EUNSUPPORTED for other sides), FUSED_QUAD is
 * CIL_EUNSUPPORTED.  FP32: polish must be 0 (no FP64 continuation; a solve
 * that reaches the FP32 floor ends with status FP32_FLOOR); polish != 0 with
 * tol > 0 is CIL_EUNSUPPORTED. */
int cil_simulate_patterns_sbdf2(cil_model model, cil_precision prec, const cil_problem *probs, int32_t B,
                                void *state, const int64_t *elem_offsets, const cil_stepping *stepping,
                                cil_solve_report *reports, void *hip_stream);

/* Simulate plans.  The paper's experiments draw every statistic from large
 * batches of independent solves of one model (Sec. 4, many initial states per
 * parameter value).  A plan binds such a batch -- problems, layout, stepping
 * and the state buffer -- to device-resident tables and solve descriptors and
 * to one instantiated HIP graph: a clear of the per-solve results, then one
 * persistent fused kernel per grid side, the sides forked over plan-owned
 * streams (default priority) and joined.  cil_sim_plan_launch replays it with
 * one graph launch, stream-ordered on the caller's stream.
 *   cil_sim_plan_create: same arguments and checks as cil_simulate_patterns;
 *     the state pointer is bound to the plan (device, caller-owned, must stay
 *     valid while the plan lives).  Every grid side must have a fused stepper
 *     (FP32 n in {32, 64, 128}, FP64 n in {32, 64}), else CIL_EUNSUPPORTED;
 *     path PLAIN gives CIL_EUNSUPPORTED; an FP32 plan with tol > 0 needs
 *     polish = 0 (a solve stopping at the FP32 floor then reports status
 *     FP32_FLOOR), else CIL_EINVAL.  Allocates; synchronises `hip_stream`.
 *     *plan receives an owned handle (free with cil_sim_plan_destroy).
 *   cil_sim_plan_tune: the autotuner.  For each grid side, times every code
 *     shape of the quad-lane stepper (the 4 values of CIL_OPT_QUAD_SHAPE) on
 *     that side's solves alone from a device copy of the bound state (which it
 *     leaves unchanged): `steps` > 0 fixed steps per trial (no stop rule), or
 *     with steps = 0 the plan's own stepping (stop rule and max_steps, so the
 *     trial time is the side's real completion time).  Keeps the fastest shape
 *     per side and re-captures the graph.  CIL_EINVAL for steps < 0 or a
 *     FUSED_LINE plan.  Allocates (a state-sized scratch); synchronises.
 *   cil_sim_plan_launch: enqueues one graph launch on hip_stream: every solve
 *     starts at step 0 from what the bound state holds and runs until its stop
 *     rule fires.  Allocates nothing, does not synchronise; launches of one
 *     plan must not overlap (they share the result arrays).
 *   cil_sim_plan_report: after the last launch on hip_stream: per-solve
 *     results (steps_fp64 is 0), reports host[B] or NULL.  Synchronises.
 *     Returns CIL_ENONFINITE if a solve ended NONFINITE.
 *   cil_sim_plan_groups / cil_sim_plan_group_info: the grid sides in launch
 *     order (most work first): side n, solve count, chosen shape, and the
 *     tuning times in ms (host[CIL_QUAD_SHAPES] or NULL; 0 before tuning).
 *   cil_sim_plan_destroy: synchronises the device, frees the plan (NULL ok). */
typedef struct cil_sim_plan_s cil_sim_plan;
enum { CIL_QUAD_SHAPES = 4 };
int cil_sim_plan_create(cil_model model, cil_precision prec, const cil_problem *probs, int32_t B, void *state,
                        const int64_t *elem_offsets, const cil_stepping *stepping, void *hip_stream,
                        cil_sim_plan **plan);
int cil_sim_plan_tune(cil_sim_plan *plan, int64_t steps, void *hip_stream);
int cil_sim_plan_launch(cil_sim_plan *plan, void *hip_stream);
int cil_sim_plan_report(cil_sim_plan *plan, cil_solve_report *reports, void *hip_stream);
int cil_sim_plan_groups(const cil_sim_plan *plan);
int cil_sim_plan_group_info(const cil_sim_plan *plan, int32_t group, int32_t *n, int32_t *count, int32_t *shape,
                            double *tuned_ms);
int cil_sim_plan_destroy(cil_sim_plan *plan);

/* ------------------------------------------------------- CIL statistic */
/* Squared distances are compared with squared radii: a pair counts under
 * radius R when D < fl(R*R) (strict, eq. eCDF).  D is the canonical squared
 * distance: with d_k = fl64(a_k - b_k) (inputs converted to double), D is the
 * exact sum of the d_k^2 rounded once to double.  Fast paths (an FP64 direct
 * sum, or for FP32 sets a split-bf16x3 Gram on the matrix cores) compute an
 * approximation with a rigorous error bound; every pair whose approximation
 * is within that bound of some fl(R_m^2) is recomputed canonically, so all
 * counts are exact.  radii: host[M], > 0, strictly decreasing, M <= 255. */

/* counts[m] = #{(i,j) : D(A_i, B_j) < fl(R_m^2)}, m = 0..M-1 (the paper's
 * m = 1..M); y[m] = counts[m] / (nA nB)  (eqs. eCDF, CIL).
 *   setA device[nA][dim], setB device[nB][dim], element type by prec.
 *   counts host[M] (required); y host[M] or NULL. */
int cil_features(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                 cil_precision prec, const double *radii, int32_t M, int64_t *counts, double *y,
                 void *hip_stream);

/* Per-pair bin matrix: bins[i*nB + j] = #{m : D(A_i,B_j) < fl(R_m^2)}
 * (device uint8[nA][nB]).  counts host[M] or NULL as in cil_features. */
int cil_pair_bins(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                  cil_precision prec, const double *radii, int32_t M, uint8_t *bins,
                  int64_t *counts, void *hip_stream);

/* Smallest and largest canonical squared distance over the pairs (i, j);
 * exclude_diagonal != 0 skips i == j (requires nA == nB).  The radii of the
 * paper's experiments are fitted to this range (Sec. 2.1, Sec. 3.2). */
int cil_distance_range(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                       cil_precision prec, int32_t exclude_diagonal, double *d2min /*host*/,
                       double *d2max /*host*/, void *hip_stream);

/* Canonical squared distances of selected pairs: d2[t] = D(A_ia[t], B_jb[t]).
 * ia, jb, d2 device[npairs].  Indices are checked on the device against nA,
 * nB: a pair with an index out of range gets d2 = NaN and the call returns
 * CIL_EINVAL (the call synchronises the stream to report this). */
int cil_canonical_d2(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                     cil_precision prec, const int64_t *ia, const int64_t *jb, int64_t npairs,
                     double *d2, void *hip_stream);

/* The fast-pass approximation of every squared distance and its rigorous
 * error bound: |d2[i*nB+j] - D(A_i, B_j)| <= eps[i*nB+j].  FP64 sets: direct
 * FP64 sums; FP32 sets: split-bf16x3 Gram on the matrix cores.  These are the
 * values the counting calls classify before re-checking pairs near a radius.
 * d2, eps device double[nA][nB].  For diagnostics and tests. */
int cil_approx_d2(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                  cil_precision prec, double *d2, double *eps, void *hip_stream);

/* Radii ladder from a squared-distance range (Sec. 2.1, Sec. 3.2):
 * R_0 = sqrt(d2max), R_M = sqrt(d2min); law 0: R_m = R_0 b^-m with
 * b = (R_0/R_M)^(1/M); law 1: R_m = R_0 - m (R_0 - R_M)/M; m = 1..M.
 * Host only; radii host[M]. */
int cil_radii(double d2min, double d2max, int32_t M, int32_t law, double *radii);

/* Range, radii and bins in one call, from a single fast pass over the pairs
 * (the adaptive radii of Sec. 3.2): d2min, d2max as cil_distance_range
 * (exclude_diagonal != 0: pairs i != j only, requires nA == nB), radii
 * host[M] as cil_radii(d2min, d2max, M, law), then bins and counts of every
 * pair (diagonal included) as cil_pair_bins with those radii.  bins device
 * uint8[nA][nB] or NULL; counts host[M] or NULL.  Errors as those three calls
 * (CIL_EINVAL for a degenerate range, e.g. all distances equal). */
int cil_pair_bins_adaptive(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                           cil_precision prec, int32_t exclude_diagonal, int32_t M, int32_t law,
                           double *d2min /*host*/,
                           double *d2max /*host*/, double *radii /*host[M]*/, uint8_t *bins,
                           int64_t *counts /*host[M]*/, void *hip_stream);

/* Diagnostics of the last distance call on this thread: pairs evaluated,
 * pairs recomputed canonically, pairs whose canonical value needed the exact
 * (slow) summation.  Host only. */
int cil_last_distance_stats(int64_t *pairs, int64_t *rechecked, int64_t *exact_fallbacks);

/* ------------------------------------------- further features (Sec. 3.1) */
/* Min-max scaling of Sec. 5 (scaled pattern data): for each pattern and
 * species, s~ = (s - min) / (max - min) over the species' n x n values,
 * evaluated in FP64 and rounded once to the element type; a constant species
 * becomes 0.  patterns, out: device [count][2][n][n] of prec (may alias).
 * CIL_EINVAL for count < 0, n < 1, count > 65535. */
int cil_minmax_scale(const void *patterns, int64_t count, int32_t n, cil_precision prec, void *out,
                     void *hip_stream);

/* Derivative augmentation for the Sobolev norms of Sec. 3.1 (derivatives by
 * forward differences, h = L / (n - 1) as the grid): pattern p ([2][n][n])
 * becomes [s (2 n^2) | D_x s (2 n (n-1)) | D_y s (2 n (n-1))] with
 * D_x s[c][i][j] = (s[c][i][j+1] - s[c][i][j]) / h (j < n - 1) and
 * D_y s[c][i][j] = (s[c][i+1][j] - s[c][i][j]) / h (i < n - 1), each evaluated
 * in FP64 and rounded once to the element type.  The W^{1,2} distance of two
 * patterns is the L2 distance of their augmented vectors (the counting calls
 * above take them as pattern sets of dimension 2 n^2 + 4 n (n-1)).
 * out: device [count][2 n^2 + 4 n (n-1)].  CIL_EINVAL for n < 2, L <= 0. */
int cil_augment_patterns(const void *patterns, int64_t count, int32_t n, double L, cil_precision prec, void *out,
                         void *hip_stream);

/* Max-abs distances per segment (the L-infinity norms of Sec. 3.1): for each
 * pair and segment s = [seg_end[s-1], seg_end[s]) (seg_end[-1] = 0),
 * D[(i nB + j) nseg + s] = max_k |A_ik - B_jk| over the segment, taken over
 * fl64(|A_ik - B_jk|) -- which is the exact maximum rounded once to double
 * (rounding is monotone); 0 for an empty segment.  seg_end host[nseg],
 * non-decreasing, <= dim, 1 <= nseg <= 8.  D device double[nA][nB][nseg]. */
int cil_pair_maxabs(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim, cil_precision prec,
                    const int64_t *seg_end, int32_t nseg, double *D, void *hip_stream);

/* out[p] over D[p][0..nseg-1]: max (mode 0), left-to-right FP64 sum (mode 1),
 * or left-to-right sum of the correctly rounded square roots (mode 2):
 * W^{1,inf} and its sum variant from per-segment maxima (eqs. norm:W1inf,
 * norm:W1infprime), and the sum-of-L2 W^{1,2} variant (eq. norm:W12prime)
 * from per-segment canonical squared distances (cil_canonical_d2). */
int cil_combine_segments(const double *D, int64_t n, int32_t nseg, int32_t mode, double *out, void *hip_stream);

/* Smallest and largest of n >= 1 non-negative finite distances V (device);
 * host outputs; synchronises. */
int cil_value_range(const double *V, int64_t n, double *vmin, double *vmax, void *hip_stream);

/* Correlation sums of distances (not squared): bins[p] = #{m : V[p] <
 * radii[m]} (device uint8[n] or NULL), counts[m] = #{p : bins[p] >= m + 1}
 * (host int64[M]).  radii host[M], > 0, strictly decreasing, M <= 255
 * (a ladder for distances: cil_radii(vmin^2, vmax^2, M, law)). */
int cil_bin_values(const double *V, int64_t n, const double *radii, int32_t M, uint8_t *bins, int64_t *counts,
                   void *hip_stream);

/* Bootstrap correlation integral vectors (Alg. 2bst / Alg. 3bst step 2):
 * resample r pairs the kA rows idxA[r][*] with the kB columns idxB[r][*]
 * (repeats allowed) and counts Ycount[r][m] = #{(a,b) : bins[idxA][idxB] > m},
 * Y[r][m] = Ycount[r][m] / (kA kB).
 *   bins device uint8[nA][nB] (from cil_pair_bins); idxA device int32[n_boot][kA];
 *   idxB device int32[n_boot][kB]; Ycount device int64[n_boot][M] or NULL;
 *   Y device double[n_boot][M] or NULL.  Indices are checked on the device;
 *   an out-of-range index makes the call return CIL_EINVAL. */
int cil_bootstrap_features(const uint8_t *bins, int64_t nA, int64_t nB, int32_t M,
                           const int32_t *idxA, int32_t kA, const int32_t *idxB, int32_t kB,
                           int32_t n_boot, int64_t *Ycount, double *Y, void *hip_stream);

/* cil_bootstrap_features for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, results and errors, but the call allocates
 * nothing -- its counters, resample multiplicities and flags live in a fixed
 * 16 MiB array per device that the library holds until the process ends.
 * Sizes whose scratch would exceed it (about 8 n_boot M + 4 n_boot_32
 * ceil128(nA) + 4 n_boot nB bytes, n_boot_32 = n_boot rounded up to 32; the
 * last two terms only for M <= 32) return CIL_EINVAL before any device work.
 * Every call on a device shares that device's array and keeps the last
 * call's contents (what must start at zero is cleared by a kernel in each
 * call), so calls that overlap on one device race; synchronises the stream
 * (index check), like cil_bootstrap_features. */
int cil_bootstrap_features_noalloc(const uint8_t *bins, int64_t nA, int64_t nB, int32_t M,
                                   const int32_t *idxA, int32_t kA, const int32_t *idxB, int32_t kB,
                                   int32_t n_boot, int64_t *Ycount, double *Y, void *hip_stream);

/* Gaussian synthetic likelihood, batched over P independent problems
 * (eqs. cil:CF, cil:CF_synth): per problem p, mu = mean of the n_boot rows of
 * Y[p] (device double[P][n_boot][M]), Sigma = their covariance (1/(n_boot-1),
 * two-pass), bins whose sample variance is exactly 0 are dropped (m_eff
 * kept), Sigma = L L^T (Cholesky), z = L^-1 (y_obs[p] - mu),
 *   f[p] = |z|^2,  loglik[p] = -f/2 - sum log L_ii - (m_eff/2) log(2 pi).
 * All in FP64 on the GPU.  f, loglik device double[P]; m_eff, status device
 * int32[P] (status CIL_OK or CIL_ENOTSPD, then f = loglik = NaN). M <= 64. */
int cil_gaussian_loglik(const double *Y, int32_t P, int32_t n_boot, int32_t M,
                        const double *y_obs, double *f, double *loglik, int32_t *m_eff,
                        int32_t *status, void *hip_stream);

/* The synthetic-likelihood statistic of two pattern sets in one call
 * (Alg. 2bst: correlation integral vectors of the cross pairs and their
 * bootstrap, then the Gaussian likelihood of eqs. cil:CF, cil:CF_synth):
 *   d2min, d2max, radii, bins, counts as cil_pair_bins_adaptive (cross pairs,
 *     no diagonal exclusion);
 *   Y as cil_bootstrap_features (idxA, idxB, kA, kB, n_boot as there);
 *   y_obs[m] = counts[m] / (nA nB), the observed vector, formed on the device;
 *   f, loglik, m_eff, status as cil_gaussian_loglik for P = 1 (Y, y_obs).
 * Same results as those calls in sequence, bit for bit, with one stream
 * synchronisation, at the end, where the re-check list's length and the
 * bootstrap indices are checked (CIL_EDEVICE, CIL_EINVAL; outputs are then
 * undefined).  The radii are formed on the device (powers in double-double,
 * rounded once) and compared at the end with cil_radii's, which are the
 * call's radii.  Where the two differ (the C library's pow is not correctly
 * rounded for every argument: about one ladder in a hundred at M = 13) the
 * bins stand unless a pair lies within 2^-44 R_m^2 of a threshold that
 * differs; then the call is redone with the host's radii and one more
 * synchronisation (CIL_OPT_STAT_DEVICE_RADII).  Host: d2min, d2max, radii[M], counts[M] (or NULL).  Device:
 * bins uint8[nA][nB], Y double[n_boot][M], y_obs double[M], f, loglik
 * double[1], m_eff, status int32[1].  1 <= M <= 64, n_boot >= 2. */
int cil_statistic_adaptive(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                           cil_precision prec, int32_t M, int32_t law, const int32_t *idxA, int32_t kA,
                           const int32_t *idxB, int32_t kB, int32_t n_boot, double *d2min, double *d2max,
                           double *radii, int64_t *counts, uint8_t *bins, double *Y, double *y_obs, double *f,
                           double *loglik, int32_t *m_eff, int32_t *status, void *hip_stream);

/* Library options (host only; they apply to later calls).
 * CIL_OPT_FORCE_EXACT_SUM (value 0/1): every canonical distance is taken by
 *   the exact (slow) summation instead of the certified double-double one;
 *   for testing that path.
 * CIL_OPT_QUAD_SHAPE (value -1..3): code shape of the fused quad-lane stepper,
 *   -1 = chosen by grid side and precision (default: 1 for n = 32, else 2
 *   in FP32 and 0 in FP64); 0 = both species of a grid line in
 *   one lane, 4n threads per solve; 1 = one species per lane, 8n threads;
 *   2, 3 = shapes 0, 1 with the column-pass divisor applied in the split
 *   step's complex form (fewer operations, a larger table).  Every shape
 *   computes the same step; timing and register use differ.
 * CIL_OPT_BOOTSTRAP_GATHER (value 0/1): 1 = bootstrap counts always by the
 *   per-resample gather kernel; 0 (default) = on the matrix cores when
 *   M <= 32 and no pattern occurs more than 256 times in a resample (the
 *   gather kernel otherwise).  Both give the same exact counts.
 * CIL_OPT_GRAM_FLUSH (value 32, 64 (default), 128 or 256): number of
 *   elements the split-bf16x3 Gram accumulates in FP32 before adding into its
 *   FP64 accumulator (at least 64 with CIL_OPT_GRAM_PIPELINE = 0).  Smaller values narrow the error band (fewer canonical
 *   re-checks) and cost more accumulator additions; counts are exact either
 *   way.  CIL_EINVAL for other values.
 * CIL_OPT_GRAM_PIPELINE (value 0, 1 or 2 (default)): how the Gram stages its
 *   tiles.  0 = loads through registers into one LDS buffer; 1 = LDS-DMA
 *   loads into two buffers, the next stage in flight while the matrix cores
 *   work; 2 = as 1 with tiles handed to the XCDs in contiguous ranges.  All
 *   compute the same products in the same order (identical results).
 *   CIL_EINVAL for other values.
 * CIL_OPT_WAVE_PRIORITY (value 0, or a base b in [2, 1e6]; default 100): in
 *   residual-stopped fused runs (tol > 0) a solve sets its wavefronts' issue
 *   priority at each evaluation from its residual r: 3, 2, 1 or 0 as r/tol
 *   exceeds b^3, b^2, b or not, so that the solves with most steps to go,
 *   which set the batch's time, win the SIMDs they share.  0 = off.  Results
 *   are unchanged (priority changes timing only).  CIL_EINVAL for 1 or
 *   values outside the range.
 * CIL_OPT_POLISH_SEPARATE (value 0/1): FP32 solves with polish != 0 on the
 *   fused quad-lane path at n = 32 or 64 (default shapes) continue from their
 *   FP32 floor inside the same persistent launch (0, default); 1 = the same
 *   kernel runs twice, the FP32 phase of the whole batch, then the polish of
 *   the solves at their floor.  Both give identical results.  (Other sides
 *   always polish in FP64 steps in a launch of their own.)
 * CIL_OPT_STAT_DEVICE_RADII (value 0, 1 (default) or 2): cil_statistic_adaptive
 *   forms the radii on the device and checks them against the host's at the
 *   end (1), or on the host after reading the range back (0); 2 = as 1 with
 *   the check always failing, so that every call takes the host's radii in a
 *   second pass (for testing that path).
 * CIL_OPT_SYNC_SPIN_US (value 0..1e7, default 200000): where a call waits
 *   for its stream (to read back results), it polls the stream's progress for
 *   up to this many microseconds before a blocking wait; 0 = block at once.
 *   Polling keeps a host core busy but avoids the wake-up delay of a blocking
 *   wait, which is about as long as the statistic's short launches.  Results
 *   are unchanged.  CIL_EINVAL outside the range. */
enum { CIL_OPT_FORCE_EXACT_SUM = 1, CIL_OPT_QUAD_SHAPE = 2, CIL_OPT_BOOTSTRAP_GATHER = 3, CIL_OPT_GRAM_FLUSH = 4,
       CIL_OPT_GRAM_PIPELINE = 5, CIL_OPT_WAVE_PRIORITY = 6, CIL_OPT_POLISH_SEPARATE = 7,
       CIL_OPT_SYNC_SPIN_US = 8, CIL_OPT_STAT_DEVICE_RADII = 9 };
int cil_set_option(int32_t option, int64_t value);

/* Kernel timing.  cil_profile(1) clears the accumulators and starts timing:
 * every hot kernel launch is then bracketed by two HIP events recorded on the
 * stream it is launched on; cil_profile(2) does the same for the fused
 * stepper kernels only (no events on the statistic's short launches);
 * cil_profile(0) stops.  cil_profile_read gives the
 * number of timed launches and their total duration in milliseconds for one
 * kernel name (0 and 0.0 if none); cil_profile_names writes the timed kernel
 * names, comma-separated, NUL-terminated, into buf[len].  Reading waits for
 * the recorded events.  Host only. */
int cil_profile(int32_t enable);
int cil_profile_read(const char *name, int64_t *count, double *total_ms);
int cil_profile_names(char *buf, int64_t len);

/* Free every internal workspace, table, auxiliary stream and cached state on
 * all devices (waits for the device to be idle first).  The library stays
 * usable: later calls allocate again. */
int cil_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* CIL_H */
