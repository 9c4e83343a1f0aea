/*
 * cil_oracle.c -- plain, slow, FP64 CPU reference for the CIL hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path: in particular the implicit diffusion solve here is a banded Cholesky
 * factorisation of the stencil matrix and uses no trigonometry at all.
 *
 * What it follows (Kazarnikov et al., arXiv 2203.14742):
 *   - kinetics: Sec. 4.1, FitzHugh-Nagumo, Gierer-Meinhardt and Brusselator
 *     reaction terms and their homogeneous steady states; the source form of
 *     Gierer-Meinhardt (u_t = Lap u + a - b u + u^2/v, v_t = d Lap v + u^2 - v)
 *     is the workload definition of the 64x64 stationarity benchmark.
 *   - space: App. B.1.1, uniform grid h = L/(n-1), five-point Laplacian,
 *     Neumann condition through first-order ghost copies (v_0 = v_1,
 *     v_{n+1} = v_n on every side), giving the method-of-lines system.
 *   - time: IMEX Euler (SBDF1): the reaction is explicit and pointwise with
 *     both species taken from the old step, the diffusion is implicit,
 *     (I - dt nu Lap_h) u^{k+1} = u^k + dt F(u^k).
 *   - stationarity: L-infinity norm of the discrete time derivative
 *     (u^{k+1} - u^k)/dt over both species (Sec. 5.1 uses the L-infinity norm
 *     of the time derivative with threshold 1e-8).
 *   - correlation sum: Sec. 2.1, eq. (eCDF): pairs with ||s_i - s_j|| < R are
 *     counted.  The comparison is made on squares, D < fl(R*R), with D the
 *     canonical squared distance defined below (strict "<", so a pair at
 *     exactly the radius is not counted).
 *
 * Canonical squared distance: with d_k = fl64(a_k - b_k) (inputs converted to
 * double first), D = RN64( sum_k d_k^2 ), the exact real sum of the exact
 * squares rounded once to double.  Each square is split exactly into
 * hi + lo with an FMA; the sum of all those doubles is accumulated exactly in
 * a non-overlapping expansion (Shewchuk's exact-summation method) and rounded
 * once at the end with round-half-even.  The value therefore does not depend
 * on the order of the terms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_FHN = 0, OR_GM = 1, OR_GM_SOURCE = 2, OR_BRUSSELATOR = 3, OR_HEAT = 4 };
enum { OR_SOLVE_OK = 0, OR_SOLVE_NONFINITE = 1, OR_SOLVE_MAXSTEPS = 2 };

/* ------------------------------------------------------------------------ */
/* Kinetics, Sec. 4.1.  p[] per model:
 *   FHN          p = {mu, eps, alpha}:  f = eps (w - alpha v),  g = -v + mu w - w^3
 *   GM           p = {mu_v, mu_w}:      f = -mu_v v + v^2/w,    g = -mu_w w + v^2
 *   GM_SOURCE    p = {a, b}:            f = a - b v + v^2/w,    g = v^2 - w
 *   BRUSSELATOR  p = {A, B}:            f = A - (B+1) v + v^2 w, g = B v - v^2 w
 *   HEAT         (no reaction)          f = g = 0                                */
void oracle_kinetics(int model, const double *p, double v, double w, double *f, double *g)
{
    switch (model) {
    case OR_FHN:
        *f = p[1] * (w - p[2] * v);
        *g = -v + p[0] * w - w * w * w;
        break;
    case OR_GM:
        *f = -p[0] * v + v * v / w;
        *g = -p[1] * w + v * v;
        break;
    case OR_GM_SOURCE:
        *f = p[0] - p[1] * v + v * v / w;
        *g = v * v - w;
        break;
    case OR_BRUSSELATOR:
        *f = p[0] - (p[1] + 1.0) * v + v * v * w;
        *g = p[1] * v - v * v * w;
        break;
    default:
        *f = 0.0;
        *g = 0.0;
        break;
    }
}

/* Homogeneous steady state f(v0,w0) = g(v0,w0) = 0, Sec. 4.1:
 * FHN (0,0); GM (mu_w/mu_v, mu_w/mu_v^2); Brusselator (A, B/A).
 * Source form of GM: g = 0 gives w0 = v0^2, then f = a - b v0 + 1 = 0 gives
 * v0 = (a+1)/b.  Heat equation: any constant; returns (0,0). */
int oracle_homogeneous_state(int model, const double *p, double *v0, double *w0)
{
    switch (model) {
    case OR_FHN: *v0 = 0.0; *w0 = 0.0; return 0;
    case OR_GM: *v0 = p[1] / p[0]; *w0 = p[1] / (p[0] * p[0]); return 0;
    case OR_GM_SOURCE: *v0 = (p[0] + 1.0) / p[1]; *w0 = (*v0) * (*v0); return 0;
    case OR_BRUSSELATOR: *v0 = p[0]; *w0 = p[1] / p[0]; return 0;
    case OR_HEAT: *v0 = 0.0; *w0 = 0.0; return 0;
    default: return -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Method-of-lines right-hand side by direct stencil evaluation, App. B.1.1.
 * state = [v grid n x n row-major][w grid n x n row-major]; out same layout. */
static double lap_ghost(const double *u, int n, int i, int j, double inv_h2)
{
    double c = u[i * n + j];
    double up = (i > 0) ? u[(i - 1) * n + j] : c;       /* ghost copy */
    double dn = (i < n - 1) ? u[(i + 1) * n + j] : c;
    double lf = (j > 0) ? u[i * n + j - 1] : c;
    double rt = (j < n - 1) ? u[i * n + j + 1] : c;
    return (up + dn + lf + rt - 4.0 * c) * inv_h2;
}

void oracle_mol_rhs(int model, const double *p, const double *nu, int n, double L,
                    const double *state, double *out)
{
    double h = L / (double)(n - 1);
    double inv_h2 = 1.0 / (h * h);
    const double *v = state, *w = state + (long)n * n;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double f, g;
            oracle_kinetics(model, p, v[i * n + j], w[i * n + j], &f, &g);
            out[i * n + j] = nu[0] * lap_ghost(v, n, i, j, inv_h2) + f;
            out[(long)n * n + i * n + j] = nu[1] * lap_ghost(w, n, i, j, inv_h2) + g;
        }
}

/* ------------------------------------------------------------------------ */
/* Banded Cholesky of A = I - c * (stencil Laplacian without 1/h^2 folded),
 * i.e. A_pp = 1 + c * deg(p), A_pq = -c for the (up to four) grid
 * neighbours q of p, with c = dt * nu / h^2.  p = i*n + j.  Half bandwidth n.
 * Lb[p*(n+1) + k] holds L[p][p-k], k = 0..n. */
static double a_entry(int n, double c, long pp, long qq)
{
    int pi = (int)(pp / n), pj = (int)(pp % n);
    if (pp == qq) {
        int deg = (pi > 0) + (pi < n - 1) + (pj > 0) + (pj < n - 1);
        return 1.0 + c * deg;
    }
    int qi = (int)(qq / n), qj = (int)(qq % n);
    int di = abs(pi - qi), dj = abs(pj - qj);
    if (di + dj == 1) return -c;
    return 0.0;
}

static int band_cholesky(int n, double c, double *Lb)
{
    long N = (long)n * n;
    int w = n;
    for (long p = 0; p < N; p++) {
        long q0 = p - w < 0 ? 0 : p - w;
        for (long q = q0; q <= p; q++) {
            double s = a_entry(n, c, p, q);
            long r0 = q0 > q - w ? q0 : q - w;
            for (long r = r0; r < q; r++)
                s -= Lb[p * (w + 1) + (p - r)] * Lb[q * (w + 1) + (q - r)];
            if (q == p) {
                if (!(s > 0.0)) return -1;
                Lb[p * (w + 1)] = sqrt(s);
            } else {
                Lb[p * (w + 1) + (p - q)] = s / Lb[q * (w + 1)];
            }
        }
    }
    return 0;
}

static void band_solve(int n, const double *Lb, double *x)
{
    long N = (long)n * n;
    int w = n;
    for (long p = 0; p < N; p++) {            /* L y = b */
        double s = x[p];
        long q0 = p - w < 0 ? 0 : p - w;
        for (long q = q0; q < p; q++) s -= Lb[p * (w + 1) + (p - q)] * x[q];
        x[p] = s / Lb[p * (w + 1)];
    }
    for (long p = N - 1; p >= 0; p--) {       /* L^T x = y */
        double s = x[p];
        long q1 = p + w > N - 1 ? N - 1 : p + w;
        for (long q = p + 1; q <= q1; q++) s -= Lb[q * (w + 1) + (q - p)] * x[q];
        x[p] = s / Lb[p * (w + 1)];
    }
}

/* Solve (I - dt nu Lap_h) x = b in place for one n x n grid. */
int oracle_implicit_diffusion(int n, double L, double dt, double nu, double *x)
{
    double h = L / (double)(n - 1);
    double c = dt * nu / (h * h);
    double *Lb = (double *)malloc(sizeof(double) * (size_t)n * n * (n + 1));
    if (!Lb) return -3;
    if (band_cholesky(n, c, Lb)) { free(Lb); return -5; }
    band_solve(n, Lb, x);
    free(Lb);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* IMEX-Euler run of one solve.  state (in: initial condition, out: state after
 * the last step taken).  tol <= 0: exactly max_steps steps.  tol > 0: stop at
 * the first step s with s % check_every == 0 whose residual is < tol.  The
 * residual of step s is max over both species and all points of
 * |u^s - u^{s-1}| / dt.  A solve whose state holds a non-finite value at a
 * residual-evaluation step (every check_every steps and the last step) stops
 * there with status NONFINITE. */
int oracle_imex_run(int model, const double *p, const double *nu, int n, double L, double dt,
                    long max_steps, double tol, int check_every, double *state,
                    long *steps_taken, double *final_resid, int *status)
{
    long N = (long)n * n;
    double h = L / (double)(n - 1);
    double *Lv = (double *)malloc(sizeof(double) * (size_t)N * (n + 1));
    double *Lw = (double *)malloc(sizeof(double) * (size_t)N * (n + 1));
    double *r = (double *)malloc(sizeof(double) * (size_t)2 * N);
    if (!Lv || !Lw || !r) { free(Lv); free(Lw); free(r); return -3; }
    if (band_cholesky(n, dt * nu[0] / (h * h), Lv) || band_cholesky(n, dt * nu[1] / (h * h), Lw)) {
        free(Lv); free(Lw); free(r); return -5;
    }
    if (check_every < 1) check_every = 1;
    long s = 0;
    double resid = 0.0;
    int st = OR_SOLVE_OK;
    for (s = 1; s <= max_steps; s++) {
        for (long q = 0; q < N; q++) {        /* explicit reaction, old values */
            double f, g;
            oracle_kinetics(model, p, state[q], state[N + q], &f, &g);
            r[q] = state[q] + dt * f;
            r[N + q] = state[N + q] + dt * g;
        }
        band_solve(n, Lv, r);                 /* implicit diffusion */
        band_solve(n, Lw, r + N);
        resid = 0.0;
        int bad = 0;
        for (long q = 0; q < 2 * N; q++) {
            double dlt = fabs(r[q] - state[q]) / dt;
            if (!isfinite(r[q])) bad = 1;
            if (dlt > resid) resid = dlt;
            state[q] = r[q];
        }
        int eval = (s % check_every == 0) || (s == max_steps);
        if (eval && bad) { st = OR_SOLVE_NONFINITE; resid = NAN; break; }
        if (eval && tol > 0.0 && resid < tol) break;
    }
    if (s > max_steps) s = max_steps;
    if (st == OR_SOLVE_OK && tol > 0.0 && !(resid < tol)) st = OR_SOLVE_MAXSTEPS;
    if (steps_taken) *steps_taken = s;
    if (final_resid) *final_resid = resid;
    if (status) *status = st;
    free(Lv); free(Lw); free(r);
    return 0;
}

/* Second-order IMEX run of one solve (semi-implicit BDF2, an alternative to
 * the paper's first-order-in-time integrators): the first step is the
 * IMEX-Euler step above; every later step s takes
 *   r   = (4 u^{s-1} - u^{s-2}) / 3 + (2 dt / 3) (2 F(u^{s-1}) - F(u^{s-2}))
 *   u^s = (I - (2 dt / 3) nu Lap_h)^{-1} r
 * (BDF2 for the time derivative, the reaction extrapolated linearly to the
 * new time level, diffusion implicit at it).  Arguments, residual, stop rule
 * and status as for oracle_imex_run. */
int oracle_sbdf2_run(int model, const double *p, const double *nu, int n, double L, double dt,
                     long max_steps, double tol, int check_every, double *state,
                     long *steps_taken, double *final_resid, int *status)
{
    long N = (long)n * n;
    double h = L / (double)(n - 1);
    double *E1 = (double *)malloc(sizeof(double) * (size_t)N * (n + 1));   /* Euler factors */
    double *E2 = (double *)malloc(sizeof(double) * (size_t)N * (n + 1));
    double *B1 = (double *)malloc(sizeof(double) * (size_t)N * (n + 1));   /* BDF2 factors */
    double *B2 = (double *)malloc(sizeof(double) * (size_t)N * (n + 1));
    double *r = (double *)malloc(sizeof(double) * (size_t)2 * N);
    double *uold = (double *)malloc(sizeof(double) * (size_t)2 * N);       /* u^{s-2} */
    double *fold = (double *)malloc(sizeof(double) * (size_t)2 * N);       /* F(u^{s-2}) */
    int rc = 0;
    if (!E1 || !E2 || !B1 || !B2 || !r || !uold || !fold) rc = -3;
    if (!rc && (band_cholesky(n, dt * nu[0] / (h * h), E1) || band_cholesky(n, dt * nu[1] / (h * h), E2) ||
                band_cholesky(n, (2.0 * dt / 3.0) * nu[0] / (h * h), B1) ||
                band_cholesky(n, (2.0 * dt / 3.0) * nu[1] / (h * h), B2)))
        rc = -5;
    if (rc) { free(E1); free(E2); free(B1); free(B2); free(r); free(uold); free(fold); return rc; }
    if (check_every < 1) check_every = 1;
    long s = 0;
    double resid = 0.0;
    int st = OR_SOLVE_OK;
    for (s = 1; s <= max_steps; s++) {
        for (long q = 0; q < N; q++) {
            double f, g;
            oracle_kinetics(model, p, state[q], state[N + q], &f, &g);
            if (s == 1) {
                r[q] = state[q] + dt * f;
                r[N + q] = state[N + q] + dt * g;
            } else {
                r[q] = (4.0 * state[q] - uold[q]) / 3.0 + (2.0 * dt / 3.0) * (2.0 * f - fold[q]);
                r[N + q] = (4.0 * state[N + q] - uold[N + q]) / 3.0 + (2.0 * dt / 3.0) * (2.0 * g - fold[N + q]);
            }
            uold[q] = state[q];
            uold[N + q] = state[N + q];
            fold[q] = f;
            fold[N + q] = g;
        }
        band_solve(n, s == 1 ? E1 : B1, r);
        band_solve(n, s == 1 ? E2 : B2, r + N);
        resid = 0.0;
        int bad = 0;
        for (long q = 0; q < 2 * N; q++) {
            double dlt = fabs(r[q] - state[q]) / dt;
            if (!isfinite(r[q])) bad = 1;
            if (dlt > resid) resid = dlt;
            state[q] = r[q];
        }
        int eval = (s % check_every == 0) || (s == max_steps);
        if (eval && bad) { st = OR_SOLVE_NONFINITE; resid = NAN; break; }
        if (eval && tol > 0.0 && resid < tol) break;
    }
    if (s > max_steps) s = max_steps;
    if (st == OR_SOLVE_OK && tol > 0.0 && !(resid < tol)) st = OR_SOLVE_MAXSTEPS;
    if (steps_taken) *steps_taken = s;
    if (final_resid) *final_resid = resid;
    if (status) *status = st;
    free(E1); free(E2); free(B1); free(B2); free(r); free(uold); free(fold);
    return 0;
}

/* Batch of independent solves (OpenMP over solves).  Per solve b: grid side
 * n[b], domain length L[b], nu[2b..2b+1], params p[4b..4b+3]; its state is at
 * element offset off[b] of state[]. */
static int imex_batch(int scheme, int model, int B, const int *n, const double *L, const double *nu,
                      const double *p, double dt, long max_steps, double tol, int check_every,
                      double *state, const long *off, long *steps_taken, double *final_resid,
                      int *status, int nthreads)
{
    int err = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : err)
#endif
    for (int b = 0; b < B; b++) {
        int rc = (scheme ? oracle_sbdf2_run : oracle_imex_run)(
            model, p + 4 * b, nu + 2 * b, n[b], L[b], dt, max_steps, tol, check_every, state + off[b],
            steps_taken ? steps_taken + b : 0, final_resid ? final_resid + b : 0, status ? status + b : 0);
        if (rc) err |= 1;
    }
    return err ? -1 : 0;
}

int oracle_imex_batch(int model, int B, const int *n, const double *L, const double *nu,
                      const double *p, double dt, long max_steps, double tol, int check_every,
                      double *state, const long *off, long *steps_taken, double *final_resid,
                      int *status, int nthreads)
{
    return imex_batch(0, model, B, n, L, nu, p, dt, max_steps, tol, check_every, state, off, steps_taken,
                      final_resid, status, nthreads);
}

/* The same batch with the second-order stepper (oracle_sbdf2_run). */
int oracle_sbdf2_batch(int model, int B, const int *n, const double *L, const double *nu,
                       const double *p, double dt, long max_steps, double tol, int check_every,
                       double *state, const long *off, long *steps_taken, double *final_resid,
                       int *status, int nthreads)
{
    return imex_batch(1, model, B, n, L, nu, p, dt, max_steps, tol, check_every, state, off, steps_taken,
                      final_resid, status, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Exact summation: a non-overlapping expansion of doubles (increasing
 * magnitude) whose exact sum is the running total. */
typedef struct { double t[96]; int m; } expansion;

static void exp_add(expansion *e, double x)
{
    int k = 0;
    for (int i = 0; i < e->m; i++) {
        double y = e->t[i];
        if (fabs(x) < fabs(y)) { double tmp = x; x = y; y = tmp; }
        double hi = x + y;
        double lo = y - (hi - x);           /* exact: |x| >= |y| */
        if (lo != 0.0) e->t[k++] = lo;
        x = hi;
    }
    e->t[k++] = x;
    e->m = k;
}

/* Round the exact expansion value once to double (half to even). */
static double exp_round(const expansion *e)
{
    int m = e->m;
    if (m == 0) return 0.0;
    double hi = e->t[--m];
    double lo = 0.0;
    while (m > 0) {
        double x = hi;
        double y = e->t[--m];
        hi = x + y;
        double yr = hi - x;
        lo = y - yr;
        if (lo != 0.0) break;
    }
    /* hi + lo is exact; if lo is exactly half an ulp of hi, the remaining
     * (smaller) terms decide the direction of rounding. */
    if (m > 0 && ((lo < 0.0 && e->t[m - 1] < 0.0) || (lo > 0.0 && e->t[m - 1] > 0.0))) {
        double y = lo * 2.0;
        double x = hi + y;
        double yr = x - hi;
        if (y == yr) hi = x;
    }
    return hi;
}

static double canonical_d2_core(const double *a64, const float *a32, const double *b64,
                                const float *b32, long d)
{
    expansion e;
    e.m = 0;
    for (long k = 0; k < d; k++) {
        double ak = a64 ? a64[k] : (double)a32[k];
        double bk = b64 ? b64[k] : (double)b32[k];
        double dk = ak - bk;
        double sq = dk * dk;
        double err = fma(dk, dk, -sq);     /* exact: dk*dk = sq + err */
        exp_add(&e, sq);
        if (err != 0.0) exp_add(&e, err);
    }
    return exp_round(&e);
}

double oracle_canonical_d2_f64(const double *a, const double *b, long d)
{
    return canonical_d2_core(a, 0, b, 0, d);
}

double oracle_canonical_d2_f32(const float *a, const float *b, long d)
{
    return canonical_d2_core(0, a, 0, b, d);
}

/* Exact sum of an arbitrary array of doubles, rounded once (used to pin the
 * expansion against an independent exact summation). */
double oracle_exact_sum(const double *x, long n)
{
    expansion e;
    e.m = 0;
    for (long k = 0; k < n; k++) exp_add(&e, x[k]);
    return exp_round(&e);
}

/* All pair distances D[i*nB + j] = canonical D(A_i, B_j).  is_f32 selects the
 * element type of both sets; rows are contiguous with stride dim. */
void oracle_pair_d2(const void *A, long nA, const void *B, long nB, long dim, int is_f32,
                    double *D, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (long i = 0; i < nA; i++)
        for (long j = 0; j < nB; j++) {
            if (is_f32)
                D[i * nB + j] = oracle_canonical_d2_f32((const float *)A + i * dim,
                                                        (const float *)B + j * dim, dim);
            else
                D[i * nB + j] = oracle_canonical_d2_f64((const double *)A + i * dim,
                                                        (const double *)B + j * dim, dim);
        }
}

/* Selected pairs only: D[t] = canonical D(A_{ia[t]}, B_{jb[t]}). */
void oracle_pair_d2_sampled(const void *A, const void *B, long dim, int is_f32, const long *ia,
                            const long *jb, long npairs, double *D, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (long t = 0; t < npairs; t++) {
        if (is_f32)
            D[t] = oracle_canonical_d2_f32((const float *)A + ia[t] * dim,
                                           (const float *)B + jb[t] * dim, dim);
        else
            D[t] = oracle_canonical_d2_f64((const double *)A + ia[t] * dim,
                                           (const double *)B + jb[t] * dim, dim);
    }
}

/* ------------------------------------------------------------------------ */
/* Correlation sums, eq. (eCDF)/(CIL): counts[m] = #{pairs : D < fl(R_m*R_m)},
 * m = 0..M-1 (the paper's m = 1..M). */
void oracle_counts(const double *D, long npairs, const double *radii, int M, int64_t *counts)
{
    for (int m = 0; m < M; m++) {
        double r2 = radii[m] * radii[m];
        int64_t c = 0;
        for (long t = 0; t < npairs; t++)
            if (D[t] < r2) c++;
        counts[m] = c;
    }
}

/* Per pair, the number of radii the pair falls under: #{m : D < fl(R_m^2)}. */
void oracle_bins(const double *D, long npairs, const double *radii, int M, uint8_t *bins)
{
    for (long t = 0; t < npairs; t++) {
        int c = 0;
        for (int m = 0; m < M; m++)
            if (D[t] < radii[m] * radii[m]) c++;
        bins[t] = (uint8_t)c;
    }
}

/* Bootstrap correlation integral vectors (Alg. 2bst step 2 / Alg. 3bst step 2):
 * resample r uses the kA rows idxA[r*kA + a] of the first set and the kB rows
 * idxB[r*kB + b] of the second set (repetitions allowed); its vector is
 * Y[r*M + m] = #{(a,b) : D[idxA, idxB] < R_m^2} / (kA * kB). */
void oracle_bootstrap(const double *D, long nB, const int32_t *idxA, int kA,
                      const int32_t *idxB, int kB, int n_boot, const double *radii, int M,
                      int64_t *Ycount, double *Y, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int r = 0; r < n_boot; r++) {
        for (int m = 0; m < M; m++) {
            double r2 = radii[m] * radii[m];
            int64_t c = 0;
            for (int a = 0; a < kA; a++) {
                long i = idxA[(long)r * kA + a];
                for (int b = 0; b < kB; b++) {
                    long j = idxB[(long)r * kB + b];
                    if (D[i * nB + j] < r2) c++;
                }
            }
            if (Ycount) Ycount[(long)r * M + m] = c;
            if (Y) Y[(long)r * M + m] = (double)c / ((double)kA * (double)kB);
        }
    }
}
