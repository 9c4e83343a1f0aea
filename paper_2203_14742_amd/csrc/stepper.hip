// Batched IMEX-Euler reaction-diffusion stepper (App. B.1.1 method-of-lines
// system of the Sec. 4.1 models) on gfx950.
//
// One step of one solve, both species s in {v, w}:
//   r_s   = u_s + dt F_s(u_v, u_w)                   (explicit, old values)
//   u_s'  = (I - dt nu_s Lap_h)^{-1} r_s              (implicit diffusion)
// Lap_h is the five-point Laplacian with ghost-copy Neumann boundaries; its
// eigenvectors are the cosine modes cos(pi k (i+1/2)/n) with eigenvalues
// -(4/h^2)(sin^2(pi k/2n) + sin^2(pi l/2n)), so the solve is: 2D DCT-II,
// divide by 1 + dt nu_s Lambda_kl, inverse 2D DCT.
//
// Two back-ends:
//   plain  one kernel per stage (reaction, row DCT, column DCT + divide,
//          column inverse, row inverse + residual), dense cosine matrices,
//          state streamed through HBM, host-driven step loop; any n >= 2.
//   fused  one persistent workgroup per solve, the whole n x n x 2 state
//          resident in LDS from the first step to the last; every line
//          transformed in registers by one lane (dct_reg.hpp) or a quad of
//          lanes (dct_quad.hpp); the workgroup evaluates its own stop rule
//          and retires; n in {32, 64, 128} (FP32), {32, 64} (FP64).
// Both evaluate the stationarity residual max |u^s - u^{s-1}| / dt in FP64
// every check_every steps (and at max_steps), per solve.  FP32 solves whose
// residual falls below the FP32 floor continue in FP64 (phase 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "cil_internal.hpp"
#include "dct_reg.hpp"
#include "stepper_common.hpp"

namespace cil {

__global__ void k_clear_results(const int *list, int nlist, StepResults R)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nlist) {
        int b = list[t];
        R.resid[b] = 0ull;
        R.maxabs[b] = 0ull;
        R.bad[b] = 0;
    }
}

// ======================================================================
// Plain back-end.  Work buffers are [slot][2][n][n] in T.  Tables per n:
// C[k][j] = cos(pi k (2j+1)/2n), Ct = C^T, Cw[k][j] = w_k C[k][j] with
// w_0 = 1/n, w_k = 2/n (so Cw^T inverts C), lam[k] = 4 sin^2(pi k/2n).

template <typename T>
__global__ void k_plain_reaction(const DevSolve *S, const int *list, const T *state, T *R,
                                 int n, int model, double dt)
{
    const int slot = blockIdx.y;
    const DevSolve s = S[list[slot]];
    const int N2 = n * n;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N2) return;
    const T *u = state + s.off;
    T *r = R + (size_t)slot * 2 * N2;
    T p[4] = {T(s.p[0]), T(s.p[1]), T(s.p[2]), T(s.p[3])};
    const T v = u[q], w = u[N2 + q];
    dispatch_model(model, [&](auto MD) {
        T f, g;
        kinetics<MD>(p, v, w, f, g);
        r[q] = v + T(dt) * f;
        r[N2 + q] = w + T(dt) * g;
    });
}

// Second-order IMEX reaction stage (semi-implicit BDF2): with the history
// uh = u^{s-2}, fh = F(u^{s-2}) (same layout as the state),
//   r = (4 u^{s-1} - u^{s-2}) / 3 + (2 dt / 3) (2 F(u^{s-1}) - F(u^{s-2})),
// followed by the diffusion solve with 2 dt / 3 in place of dt.  The first
// step of a call is the IMEX-Euler stage (no history yet).  Either way the
// history moves on to u^{s-1}, F(u^{s-1}).
template <typename T>
__global__ void k_plain_reaction_sbdf2(const DevSolve *S, const int *list, const T *state, T *R, T *uh, T *fh,
                                       int n, int model, double dt, int first)
{
    const int slot = blockIdx.y;
    const DevSolve s = S[list[slot]];
    const int N2 = n * n;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N2) return;
    const T *u = state + s.off;
    T *up = uh + s.off, *fp = fh + s.off;
    T *r = R + (size_t)slot * 2 * N2;
    T p[4] = {T(s.p[0]), T(s.p[1]), T(s.p[2]), T(s.p[3])};
    const T v = u[q], w = u[N2 + q];
    dispatch_model(model, [&](auto MD) {
        T f, g;
        kinetics<MD>(p, v, w, f, g);
        if (first) {
            r[q] = v + T(dt) * f;
            r[N2 + q] = w + T(dt) * g;
        } else {
            const T c = T(2.0 * dt / 3.0), third = T(1.0 / 3.0);
            r[q] = (T(4) * v - up[q]) * third + c * (T(2) * f - fp[q]);
            r[N2 + q] = (T(4) * w - up[N2 + q]) * third + c * (T(2) * g - fp[N2 + q]);
        }
        up[q] = v;
        up[N2 + q] = w;
        fp[q] = f;
        fp[N2 + q] = g;
    });
}

// out[i][l] = sum_j in[i][j] C[l][j]   (row forward)
template <typename T>
__global__ void k_plain_rows_fwd(const int *list, const T *in, T *out, const T *Ct, int n)
{
    const int slot = blockIdx.y;
    const int N2 = n * n;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * N2) return;
    (void)list;
    const int sp = e / N2, i = (e / n) % n, l = e % n;
    const T *x = in + (size_t)slot * 2 * N2 + (size_t)sp * N2 + (size_t)i * n;
    T acc = T(0);
    #pragma unroll 8
    for (int j = 0; j < n; ++j) acc += x[j] * Ct[j * n + l];
    out[(size_t)slot * 2 * N2 + e] = acc;
}

// out[k][l] = S_kl * sum_i C[k][i] in[i][l],  S_kl = 1/(1 + dt nu (lam_k+lam_l)/h^2)
template <typename T>
__global__ void k_plain_cols_fwd_div(const DevSolve *S, const int *list, const T *in, T *out,
                                     const T *C, const double *lam, int n, double dt)
{
    const int slot = blockIdx.y;
    const DevSolve s = S[list[slot]];
    const int N2 = n * n;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * N2) return;
    const int sp = e / N2, k = (e / n) % n, l = e % n;
    const T *x = in + (size_t)slot * 2 * N2 + (size_t)sp * N2;
    T acc = T(0);
    #pragma unroll 8
    for (int i = 0; i < n; ++i) acc += C[k * n + i] * x[i * n + l];
    const double nu = sp ? s.nu[1] : s.nu[0];     // a select: an indexed read would place s in memory
    const double fac = 1.0 / (1.0 + dt * nu * (lam[k] + lam[l]) * s.inv_h2);
    out[(size_t)slot * 2 * N2 + e] = acc * T(fac);
}

// out[i][l] = sum_k Cw[k][i] in[k][l]   (column inverse)
template <typename T>
__global__ void k_plain_cols_inv(const int *list, const T *in, T *out, const T *Cw, int n)
{
    const int slot = blockIdx.y;
    (void)list;
    const int N2 = n * n;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * N2) return;
    const int sp = e / N2, i = (e / n) % n, l = e % n;
    const T *x = in + (size_t)slot * 2 * N2 + (size_t)sp * N2;
    T acc = T(0);
    #pragma unroll 8
    for (int k = 0; k < n; ++k) acc += Cw[k * n + i] * x[k * n + l];
    out[(size_t)slot * 2 * N2 + e] = acc;
}

// u'[i][j] = sum_l in[i][l] Cw[l][j]   (row inverse), written to the state;
// at an evaluation step also the residual against the old state.
template <typename T>
__global__ void k_plain_rows_inv(const DevSolve *S, const int *list, const T *in, T *state,
                                 const T *Cw, int n, int check, StepResults R)
{
    const int slot = blockIdx.y;
    const int b = list[slot];
    const DevSolve s = S[b];
    const int N2 = n * n;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0, a = 0.0;
    int bad = 0;
    if (e < 2 * N2) {
        const int sp = e / N2, i = (e / n) % n, j = e % n;
        const T *x = in + (size_t)slot * 2 * N2 + (size_t)sp * N2 + (size_t)i * n;
        T acc = T(0);
        #pragma unroll 8
        for (int l = 0; l < n; ++l) acc += x[l] * Cw[l * n + j];
        T *u = state + s.off;
        if (check) {
            const double old = (double)u[e];
            d = fabs((double)acc - old);
            a = fabs((double)acc);
            bad = !isfinite((double)acc);
        }
        u[e] = acc;
    }
    if (check) {
        d = wave_max(isnan(d) ? 0.0 : d);
        a = wave_max(isnan(a) ? 0.0 : a);
        bad = wave_or(bad);
        if ((threadIdx.x & 63) == 0) {
            atomicMax(&R.resid[b], (unsigned long long)__double_as_longlong(d));
            atomicMax(&R.maxabs[b], (unsigned long long)__double_as_longlong(a));
            if (bad) atomicOr(&R.bad[b], 1);
        }
    }
}

// ======================================================================
// Fused back-end: one workgroup per solve, both species resident in LDS as
// u[2][N][N+1] (padded rows).  The workgroup runs its solve by itself: at
// every evaluation step (a multiple of check_every, or max_steps) it keeps
// the previous state in HBM, takes the step, computes the FP64 residual
// max |u^s - u^{s-1}| / dt, max |u| and a non-finite flag over both species,
// and retires when the stop rule fires.  No host round trip per step.


template <int N>
__device__ __forceinline__ int lds_addr(int e)
{
    const int c = e / (N * N), rem = e % (N * N);
    return c * (N * (N + 1)) + (rem / N) * (N + 1) + rem % N;
}

// Load the solve, step it with body() (one IMEX step on the LDS state,
// ending with a barrier) until the stop rule fires, store it.
template <typename T, int N, int THREADS, typename Body>
__device__ __forceinline__ void run_solve(T *sm, T *u, int b, double dt, const PersistArgs &pa, Body &&body)
{
    constexpr int WAVES = THREADS / 64;
    __shared__ double red[2 * WAVES];
    __shared__ int s_bad;
    __shared__ int s_stop;
    const int tid = threadIdx.x;
    for (int e = tid; e < 2 * N * N; e += THREADS) sm[lds_addr<N>(e)] = u[e];
    if (tid == 0) s_bad = 0;
    __syncthreads();
    long long step = pa.steps[b];
    while (step < pa.max_steps) {
        const long long next = step + 1;
        const bool eval = (next % pa.check == 0) || (next == pa.max_steps);
        if (eval)
            for (int e = tid; e < 2 * N * N; e += THREADS) u[e] = sm[lds_addr<N>(e)];
        body();
        step = next;
        if (eval) {
            double d = 0.0, a = 0.0;
            int bad = 0;
            for (int e = tid; e < 2 * N * N; e += THREADS) {
                const T nv = sm[lds_addr<N>(e)];
                const double dv = fabs((double)nv - (double)u[e]);
                const double av = fabs((double)nv);
                if (!isfinite((double)nv)) bad = 1;
                d = fmax(d, isnan(dv) ? 0.0 : dv);
                a = fmax(a, isnan(av) ? 0.0 : av);
            }
            d = wave_max(d);
            a = wave_max(a);
            bad = wave_or(bad);
            const int wv = tid / 64;
            if ((tid & 63) == 0) {
                red[wv] = d;
                red[WAVES + wv] = a;
                if (bad) s_bad = 1;
            }
            __syncthreads();
            if (tid == 0) {
                double dm = 0.0, am = 0.0;
                for (int w = 0; w < WAVES; ++w) {
                    dm = fmax(dm, red[w]);
                    am = fmax(am, red[WAVES + w]);
                }
                const double r = dm / dt;
                int st = -1;
                if (s_bad) st = CIL_SOLVE_NONFINITE;
                else if (pa.tol > 0.0 && r < pa.tol) st = CIL_SOLVE_OK;
                else if (pa.tol > 0.0 && pa.floor_coef > 0.0 && r < pa.floor_coef * am) st = CIL_SOLVE_FP32_FLOOR;
                else if (next == pa.max_steps) st = pa.tol > 0.0 ? CIL_SOLVE_MAXSTEPS : CIL_SOLVE_OK;
                pa.resid[b] = s_bad ? (double)NAN : r;
                if (st >= 0) pa.status[b] = st;
                s_stop = st >= 0;
            }
            __syncthreads();
            if (s_stop) break;
        }
    }
    for (int e = tid; e < 2 * N * N; e += THREADS) u[e] = sm[lds_addr<N>(e)];
    if (tid == 0) pa.steps[b] = step;
}

// Line variant: 2N threads, thread t handles species t / N, line t % N,
// whole line in its registers (dct_reg.hpp).
template <typename T, int N>
__global__ __launch_bounds__(2 * N) void k_fused(const DevSolve *S, const int *list, T *state, const T *tables,
                                                 int model, double dt, PersistArgs pa)
{
    using D = DctLine<T, N>;
    constexpr int LD = N + 1, SP = N * LD, THREADS = 2 * N;
    __shared__ T sm[2 * SP];
    const int b = list[blockIdx.x];
    const DevSolve s = S[b];
    T *u = state + s.off;
    const T *tab = tables + (size_t)s.tab * 2 * N * N;
    const int tid = threadIdx.x;
    const int sp = tid / N, ln = tid % N;
    T p[4] = {T(s.p[0]), T(s.p[1]), T(s.p[2]), T(s.p[3])};
    const T tdt = T(dt);
    T *ms = sm + sp * SP;
    run_solve<T, N, THREADS>(sm, u, b, dt, pa, [&]() {
        dispatch_model(model, [&](auto MD) {        // explicit reaction, pointwise
            for (int q = tid; q < N * N; q += THREADS) {
                const int a = (q / N) * LD + q % N;
                const T v = sm[a], w = sm[SP + a];
                T f, g;
                kinetics<MD>(p, v, w, f, g);
                sm[a] = v + tdt * f;
                sm[SP + a] = w + tdt * g;
            }
        });
        __syncthreads();
        {   // forward DCT along rows
            T x[N], X[N];
#pragma unroll
            for (int j = 0; j < N; ++j) x[j] = ms[ln * LD + j];
            D::forward(x, X);
#pragma unroll
            for (int j = 0; j < N; ++j) ms[ln * LD + j] = X[j];
        }
        __syncthreads();
        {   // forward along columns, spectral divide, inverse along columns
            T x[N], X[N];
#pragma unroll
            for (int i = 0; i < N; ++i) x[i] = ms[i * LD + ln];
            D::forward(x, X);
            const T *tb = tab + (size_t)sp * N * N + ln;
#pragma unroll
            for (int k = 0; k < N; ++k) X[k] *= tb[k * N];
            D::inverse(X, x);
#pragma unroll
            for (int i = 0; i < N; ++i) ms[i * LD + ln] = x[i];
        }
        __syncthreads();
        {   // inverse along rows
            T x[N], X[N];
#pragma unroll
            for (int j = 0; j < N; ++j) X[j] = ms[ln * LD + j];
            D::inverse(X, x);
#pragma unroll
            for (int j = 0; j < N; ++j) ms[ln * LD + j] = x[j];
        }
        __syncthreads();
    });
}

// Second-order line variant (semi-implicit BDF2): as k_fused, with the
// history u^{s-2}, F(u^{s-2}) resident in LDS beside the state.  The first
// step of the launch is the IMEX-Euler step (tables tabE, built with dt);
// later steps take r = (4 u^{s-1} - u^{s-2}) / 3 + (2 dt / 3)(2 F(u^{s-1}) -
// F(u^{s-2})) and the diffusion solve with 2 dt / 3 (tables tabB).
template <typename T, int N>
__global__ __launch_bounds__(2 * N) void k_fused_sbdf2(const DevSolve *S, const int *list, T *state, const T *tabE,
                                                       const T *tabB, int model, double dt, PersistArgs pa)
{
    using D = DctLine<T, N>;
    constexpr int LD = N + 1, SP = N * LD, THREADS = 2 * N;
    __shared__ T sm[6 * SP];                       // state [2][N][N+1], then u^{s-2}, then F(u^{s-2})
    T *uh = sm + 2 * SP, *fh = sm + 4 * SP;
    const int b = list[blockIdx.x];
    const DevSolve s = S[b];
    T *u = state + s.off;
    const size_t toff = (size_t)s.tab * 2 * N * N;
    const int tid = threadIdx.x;
    const int sp = tid / N, ln = tid % N;
    T p[4] = {T(s.p[0]), T(s.p[1]), T(s.p[2]), T(s.p[3])};
    const T tdt = T(dt), c23 = T(2.0 * dt / 3.0), third = T(1.0 / 3.0);   // a multiply, not a divide
    T *ms = sm + sp * SP;
    bool first = true;
    run_solve<T, N, THREADS>(sm, u, b, dt, pa, [&]() {
        dispatch_model(model, [&](auto MD) {        // reaction stage, pointwise
            for (int q = tid; q < N * N; q += THREADS) {
                const int a = (q / N) * LD + q % N;
                const T v = sm[a], w = sm[SP + a];
                T f, g;
                kinetics<MD>(p, v, w, f, g);
                if (first) {
                    sm[a] = v + tdt * f;
                    sm[SP + a] = w + tdt * g;
                } else {
                    sm[a] = (T(4) * v - uh[a]) * third + c23 * (T(2) * f - fh[a]);
                    sm[SP + a] = (T(4) * w - uh[SP + a]) * third + c23 * (T(2) * g - fh[SP + a]);
                }
                uh[a] = v;
                uh[SP + a] = w;
                fh[a] = f;
                fh[SP + a] = g;
            }
        });
        __syncthreads();
        {   // forward DCT along rows
            T x[N], X[N];
#pragma unroll
            for (int j = 0; j < N; ++j) x[j] = ms[ln * LD + j];
            D::forward(x, X);
#pragma unroll
            for (int j = 0; j < N; ++j) ms[ln * LD + j] = X[j];
        }
        __syncthreads();
        {   // forward along columns, spectral divide, inverse along columns
            T x[N], X[N];
#pragma unroll
            for (int i = 0; i < N; ++i) x[i] = ms[i * LD + ln];
            D::forward(x, X);
            const T *tb = (first ? tabE : tabB) + toff + (size_t)sp * N * N + ln;
#pragma unroll
            for (int k = 0; k < N; ++k) X[k] *= tb[k * N];
            D::inverse(X, x);
#pragma unroll
            for (int i = 0; i < N; ++i) ms[i * LD + ln] = x[i];
        }
        __syncthreads();
        {   // inverse along rows
            T x[N], X[N];
#pragma unroll
            for (int j = 0; j < N; ++j) X[j] = ms[ln * LD + j];
            D::inverse(X, x);
#pragma unroll
            for (int j = 0; j < N; ++j) ms[ln * LD + j] = x[j];
        }
        __syncthreads();
        first = false;
    });
}

// Spectral tables for the fused back-end:
// tab[s][k][l] = 1 / (4 N^2 (1 + dt nu_s (lam_k + lam_l) / h^2)), in FP64 then T.
struct TabSpec {
    double inv_h2, nu0, nu1;
};
template <typename T>
__global__ void k_make_tables(const TabSpec *specs, int ntab, int n, double dt, T *out)
{
    const int t = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntab || e >= 2 * n * n) return;
    const int sp = e / (n * n), k = (e / n) % n, l = e % n;
    const TabSpec ts = specs[t];
    const double sk = sinpi((double)k / (2.0 * n)), sl = sinpi((double)l / (2.0 * n));
    const double lam = 4.0 * (sk * sk + sl * sl) * ts.inv_h2;
    const double nu = sp ? ts.nu1 : ts.nu0;
    out[(size_t)t * 2 * n * n + e] = T(1.0 / (4.0 * n * (double)n * (1.0 + dt * nu * lam)));
}

// Quad-variant table: the column pass applies the divisor in the split
// step's V form.  With Y = X_k - i X_{N-k} = ph V (ph = exp(-i pi k / 2N)),
// dividing X_k by D_k and X_{N-k} by D_{N-k} is Y' = S Y + Delta conj(Y),
// S = (D_k + D_{N-k}) / 2, Delta = (D_k - D_{N-k}) / 2, so
// V' = S V + Delta exp(i pi k / N) conj(V):
//   Re V' = A Re V + Ci Im V,  Im V' = B Im V + Ci Re V,
//   A = S + Delta cos(pi k/N), B = S - Delta cos(pi k/N), Ci = Delta sin(pi k/N).
// k = 0 keeps only Re V (X_N does not exist): A = D_0, B = Ci = 0.  Row k = M
// of plane A holds D_M (X_M is carried as a real value).
// Layout: vt[t][s][plane A|B|Ci][k = 0..M][l], M = n/2 (D indexed as tab above).
template <typename T>
__global__ void k_make_vtables(const TabSpec *specs, int ntab, int n, double dt, T *out)
{
    const int t = blockIdx.y;
    const int M = n / 2, rows = M + 1;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntab || e >= 2 * rows * n) return;
    const int sp = e / (rows * n), k = (e / n) % rows, l = e % n;
    const TabSpec ts = specs[t];
    const double nu = sp ? ts.nu1 : ts.nu0;
    auto D = [&](int kk) {
        const double sk = sinpi((double)kk / (2.0 * n)), sl = sinpi((double)l / (2.0 * n));
        const double lam = 4.0 * (sk * sk + sl * sl) * ts.inv_h2;
        return 1.0 / (4.0 * n * (double)n * (1.0 + dt * nu * lam));
    };
    double A, B = 0.0, C = 0.0;
    if (k == 0 || k == M) {
        A = D(k);
    } else {
        const double dk = D(k), dn = D(n - k);
        const double S = 0.5 * (dk + dn), Dl = 0.5 * (dk - dn);
        double sn, cs;
        sincospi((double)k / n, &sn, &cs);
        A = S + Dl * cs;
        B = S - Dl * cs;
        C = Dl * sn;
    }
    T *o = out + (size_t)t * 2 * 3 * rows * n + (size_t)sp * 3 * rows * n + (size_t)k * n + l;
    o[0] = T(A);
    o[(size_t)rows * n] = T(B);
    o[(size_t)2 * rows * n] = T(C);
}

template <typename S, typename D>
__global__ void k_convert_solves(const DevSolve *Ssrc, const DevSolve *Sdst, const int *list,
                                 const S *src, D *dst)
{
    const int b = list[blockIdx.y];
    const DevSolve a = Ssrc[b], c = Sdst[b];
    const int sz = 2 * a.n * a.n;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < sz; e += gridDim.x * blockDim.x)
        dst[c.off + e] = D(src[a.off + e]);
}

// ======================================================================
// Host side.

namespace {

struct PlainTables {
    void *C = nullptr, *Ct = nullptr, *Cw = nullptr;   // T[n*n]
    double *lam = nullptr;                              // double[n]
};
std::map<std::tuple<int, int, int>, PlainTables> g_plain_tables;   // (device, n, is_f32)

template <typename T>
int plain_tables(int n, PlainTables *out)
{
    int dev;
    CIL_TRY(current_device(&dev));
    auto key = std::make_tuple(dev, n, (int)std::is_same<T, float>::value);
    auto it = g_plain_tables.find(key);
    if (it != g_plain_tables.end()) {
        *out = it->second;
        return CIL_OK;
    }
    std::vector<T> C(n * n), Ct(n * n), Cw(n * n);
    std::vector<double> lam(n);
    for (int k = 0; k < n; ++k) {
        const double wk = (k == 0 ? 1.0 : 2.0) / n;
        for (int j = 0; j < n; ++j) {
            const double c = std::cos(M_PI * k * (2.0 * j + 1.0) / (2.0 * n));
            C[k * n + j] = T(c);
            Ct[j * n + k] = T(c);
            Cw[k * n + j] = T(wk * c);
        }
        const double sk = std::sin(M_PI * k / (2.0 * n));
        lam[k] = 4.0 * sk * sk;
    }
    PlainTables t;
    size_t bytes = sizeof(T) * n * n;
    if (hipMalloc(&t.C, bytes) != hipSuccess || hipMalloc(&t.Ct, bytes) != hipSuccess ||
        hipMalloc(&t.Cw, bytes) != hipSuccess || hipMalloc(&t.lam, sizeof(double) * n) != hipSuccess)
        return set_error(CIL_ENOMEM, "table allocation failed");
    CIL_HIP(hipMemcpy(t.C, C.data(), bytes, hipMemcpyHostToDevice));
    CIL_HIP(hipMemcpy(t.Ct, Ct.data(), bytes, hipMemcpyHostToDevice));
    CIL_HIP(hipMemcpy(t.Cw, Cw.data(), bytes, hipMemcpyHostToDevice));
    CIL_HIP(hipMemcpy(t.lam, lam.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    g_plain_tables[key] = t;
    *out = t;
    return CIL_OK;
}

// Auxiliary streams (default priority) for running the persistent kernels of
// different grid sides side by side, and fork/join events; per device.
struct AuxStreams {
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> ev;     // ev[0] fork, ev[1 + g] join of stream g
};
std::map<int, AuxStreams> g_aux;

int aux_streams(int count, AuxStreams **out)
{
    int dev;
    CIL_TRY(current_device(&dev));
    AuxStreams &a = g_aux[dev];
    while ((int)a.st.size() < count) {
        hipStream_t s;
        CIL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        a.st.push_back(s);
    }
    while ((int)a.ev.size() < count + 1) {
        hipEvent_t e;
        CIL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        a.ev.push_back(e);
    }
    *out = &a;
    return CIL_OK;
}

int fused_supported(int n, bool f32)
{
    return f32 ? (n == 32 || n == 64 || n == 128) : (n == 32 || n == 64);
}

int g_quad_shape_option = -1;
int g_polish_separate = 0;         // 1: the polish always in a launch of its own
// 0: off, else the base of the priority levels.  Measured on the 500-solve GM
// batch (FP64, residual 1e-8): off 30.5 ms; base 3: 30.2; 10: 29.9; 100: 29.5;
// 1000: 29.4.
double g_wave_priority = 100.0;

int quad_shape(bool f32, int n)
{
    if (g_quad_shape_option >= 0) return g_quad_shape_option;
    // Measured on MI355X with the plans' autotuner (completion time of whole
    // batches): 32^2 runs fastest with one species per lane (128 FHN solves:
    // FP32 12.2 ms against 18.3 for both species per lane, FP64 16.2 against
    // 24.6); 64^2 and 128^2 with both species per lane, where the V-form
    // divisor pays in FP32 but not in FP64 (500 GM 64^2 solves in FP64: 30.4
    // ms X-form, 33.6 V-form; its third table plane costs more load latency
    // than it saves operations).
    if (n == 32) return 1;
    return f32 ? 2 : 0;
}

}  // namespace

// Device blocks reused across simulate calls, per device: a call's buffers go
// back to this pool instead of hipFree, so repeated calls of similar size
// allocate nothing.  Freed by cil_shutdown.
std::mutex g_pool_mu;
std::map<int, std::multimap<size_t, void *>> g_pool;     // device -> (capacity, block)

size_t pool_capacity(size_t bytes)
{
    if (bytes <= ((size_t)1 << 20)) {
        size_t c = 256;
        while (c < bytes) c <<= 1;
        return c;
    }
    return (bytes + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
}

// Library-owned stepper resources (cached DCT matrices of the plain path,
// auxiliary streams and events, the pool of call buffers), freed by
// cil_shutdown.
int stepper_release()
{
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_plain_tables) {
        (void)hipSetDevice(std::get<0>(kv.first));
        (void)hipFree(kv.second.C);
        (void)hipFree(kv.second.Ct);
        (void)hipFree(kv.second.Cw);
        (void)hipFree(kv.second.lam);
    }
    g_plain_tables.clear();
    for (auto &kv : g_aux) {
        (void)hipSetDevice(kv.first);
        for (hipStream_t st : kv.second.st) (void)hipStreamDestroy(st);
        for (hipEvent_t e : kv.second.ev) (void)hipEventDestroy(e);
    }
    g_aux.clear();
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (auto &kv : g_pool) {
            (void)hipSetDevice(kv.first);
            for (auto &b : kv.second) (void)hipFree(b.second);
        }
        g_pool.clear();
    }
    (void)hipSetDevice(cur);
    return CIL_OK;
}

int set_polish_separate(int64_t v)
{
    if (v != 0 && v != 1) return set_error(CIL_EINVAL, "polish option must be 0 or 1");
    g_polish_separate = (int)v;
    return CIL_OK;
}

int set_wave_priority(int64_t v)
{
    if (v < 0 || v == 1 || v > 1000000) return set_error(CIL_EINVAL, "wave priority option must be 0 or in [2, 1e6]");
    g_wave_priority = (double)v;
    return CIL_OK;
}

int set_quad_shape(int64_t v)
{
    if (v < -1 || v >= kQuadShapes) return set_error(CIL_EINVAL, "quad shape %lld out of range", (long long)v);
    g_quad_shape_option = (int)v;
    return CIL_OK;
}

namespace {

template <typename T>
int launch_persistent(int n, bool quad, int shape, int nl, const DevSolve *S, const int *list, T *state, const T *tables,
                      int model, double dt, const PersistArgs &pa, hipStream_t st)
{
    const bool f32 = std::is_same<T, float>::value;
    const int ni = n == 32 ? 0 : (n == 64 ? 1 : 2);
    static const char *nq32[3] = {"k_fused_q_f32_n32", "k_fused_q_f32_n64", "k_fused_q_f32_n128"};
    static const char *nq64[3] = {"k_fused_q_f64_n32", "k_fused_q_f64_n64", "k_fused_q_f64_n128"};
    static const char *nl32[3] = {"k_fused_f32_n32", "k_fused_f32_n64", "k_fused_f32_n128"};
    static const char *nl64[3] = {"k_fused_f64_n32", "k_fused_f64_n64", "k_fused_f64_n128"};
    const char *name = quad ? (f32 ? nq32[ni] : nq64[ni]) : (f32 ? nl32[ni] : nl64[ni]);
    if (!f32 && n == 128) return set_error(CIL_EUNSUPPORTED, "fused FP64 stepper supports n = 32, 64");
    const ProfMark pm = prof_begin(name, st);
    if (quad) {
        const int rc = f32 ? launch_quad_f32(n, shape, nl, S, list, (float *)state, (const float *)tables, model, dt, pa, st)
                           : launch_quad_f64(n, shape, nl, S, list, (double *)state, (const double *)tables, model, dt,
                                             pa, st);
        if (rc) return set_error(rc, "no fused quad kernel for n = %d", n);
    } else {
        if (n == 32)
            hipLaunchKernelGGL((k_fused<T, 32>), dim3(nl), dim3(64), 0, st, S, list, state, tables, model, dt, pa);
        else if (n == 64)
            hipLaunchKernelGGL((k_fused<T, 64>), dim3(nl), dim3(128), 0, st, S, list, state, tables, model, dt, pa);
        else if constexpr (std::is_same<T, float>::value)
            hipLaunchKernelGGL((k_fused<T, 128>), dim3(nl), dim3(256), 0, st, S, list, state, tables, model, dt, pa);
    }
    prof_end(pm, st);
    return check_launch(name);
}

// One plain group: solves with one grid side n, advanced in lockstep.
struct PlainGroup {
    int n = 0;
    std::vector<int> active;
    int *dlist = nullptr;
    void *work = nullptr;         // 2 buffers [cap][2][n][n]
    size_t work_cap = 0;
};

// History of the second-order stepper for one plain launch: u^{s-2} and
// F(u^{s-2}) in the state's layout, and the step index the launch starts at.
template <typename T>
struct Sbdf2Args {
    T *uh, *fh;
    int64_t step0;
};

template <typename T>
int launch_plain(PlainGroup &g, const DevSolve *S, T *u, int nl, int model, double dt, int K, StepResults R,
                 hipStream_t st, const Sbdf2Args<T> *bdf = nullptr)
{
    PlainTables tb;
    CIL_TRY(plain_tables<T>(g.n, &tb));
    const int n = g.n, N2 = n * n;
    T *A = (T *)g.work;
    T *Bw = A + g.work_cap * 2 * N2;
    const dim3 blk(256);
    const dim3 grid1((N2 + 255) / 256, nl), grid2((2 * N2 + 255) / 256, nl);
    const bool f32 = std::is_same<T, float>::value;
    const ProfMark pm = prof_begin(bdf ? (f32 ? "plain_step_sbdf2_f32" : "plain_step_sbdf2_f64")
                                       : (f32 ? "plain_step_f32" : "plain_step_f64"), st);
    for (int k = 0; k < K; ++k) {
        const int check = (k == K - 1);
        double dts = dt;                   // the diffusion solve's step
        if (bdf) {
            const int first = (bdf->step0 + k == 0);
            if (!first) dts = 2.0 * dt / 3.0;
            hipLaunchKernelGGL(k_plain_reaction_sbdf2<T>, grid1, blk, 0, st, S, g.dlist, u, A, bdf->uh, bdf->fh, n,
                               model, dt, first);
        } else {
            hipLaunchKernelGGL(k_plain_reaction<T>, grid1, blk, 0, st, S, g.dlist, u, A, n, model, dt);
        }
        hipLaunchKernelGGL(k_plain_rows_fwd<T>, grid2, blk, 0, st, g.dlist, A, Bw, (const T *)tb.Ct, n);
        hipLaunchKernelGGL(k_plain_cols_fwd_div<T>, grid2, blk, 0, st, S, g.dlist, Bw, A, (const T *)tb.C, tb.lam, n,
                           dts);
        hipLaunchKernelGGL(k_plain_cols_inv<T>, grid2, blk, 0, st, g.dlist, A, Bw, (const T *)tb.Cw, n);
        hipLaunchKernelGGL(k_plain_rows_inv<T>, grid2, blk, 0, st, S, g.dlist, Bw, u, (const T *)tb.Cw, n, check, R);
    }
    prof_end(pm, st);
    return check_launch("plain stepper");
}

}  // namespace

// Device buffers owned by one simulate call (returned to the pool at its end;
// a call that did not reach its final synchronisation first waits for the
// device, so no block goes back while queued work may still use it).
struct CallBuffers {
    struct Block {
        void *p;
        size_t cap;
        int dev;
    };
    std::vector<Block> blocks;
    bool done = false;
    ~CallBuffers()
    {
        if (blocks.empty()) return;
        if (!done) (void)hipDeviceSynchronize();
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (const Block &b : blocks) g_pool[b.dev].emplace(b.cap, b.p);
    }
    int alloc(void **p, size_t bytes)
    {
        int dev;
        CIL_TRY(current_device(&dev));
        const size_t cap = pool_capacity(bytes == 0 ? 16 : bytes);
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            auto &m = g_pool[dev];
            auto it = m.lower_bound(cap);
            if (it != m.end() && it->first <= 2 * cap) {
                *p = it->second;
                blocks.push_back(Block{it->second, it->first, dev});
                m.erase(it);
                return CIL_OK;
            }
        }
        if (hipMalloc(p, cap) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(CIL_ENOMEM, "device allocation of %zu bytes failed", cap);
        }
        blocks.push_back(Block{*p, cap, dev});
        return CIL_OK;
    }
};

namespace {

struct SimCtx {
    int model;
    double dt, tol;
    int64_t max_steps;
    int check;
    double floor_coef32;          // FP32 floor per unit max|u| (0 if no floor test)
    hipStream_t st;
    CallBuffers *cb;
    std::vector<int64_t> steps;   // per solve (host)
    std::vector<double> fres;
    std::vector<int> status;
    std::vector<int64_t> sw;      // mixed launches: step of the FP32 -> FP64 switch (-1: not a mixed solve)
    int polish = 0;               // 0 none, 1 FP64 steps, 2 refinement form (FP32 calls)
    int scheme = 0;               // 0 IMEX Euler, 1 second-order IMEX (plain back-end)
    void *uh = nullptr, *fh = nullptr;   // second-order history, state layout
};

// FP32 -> FP64 within one launch (k_fused_q_mixed) for these grid sides.
struct MixedArgs {
    double *state64;              // FP64 snapshots or FP64 state, same element layout as the FP32 state
    long long *sw;                // per solve: switch step
    int refine;                   // 1: the continuation is the refinement form, else FP64 steps
};

bool mixed_supported(int n, bool quad)
{
    return quad && g_quad_shape_option < 0 && (n == 32 || n == 64);
}

// Spectral tables for the solves in `ids` (side n): one per distinct (h, nu);
// sets hs[b].tab.  Returns the device table buffer.
template <typename T>
int make_tables(SimCtx &c, int n, const std::vector<int> &ids, std::vector<DevSolve> &hs, void **tables, bool vform,
                double dt_tab = 0.0)
{
    const double dtt = dt_tab > 0.0 ? dt_tab : c.dt;
    std::map<std::tuple<double, double, double>, int> uniq;
    std::vector<TabSpec> specs;
    for (int b : ids) {
        auto key = std::make_tuple(hs[b].inv_h2, hs[b].nu[0], hs[b].nu[1]);
        auto it = uniq.find(key);
        if (it == uniq.end()) {
            it = uniq.emplace(key, (int)specs.size()).first;
            specs.push_back(TabSpec{hs[b].inv_h2, hs[b].nu[0], hs[b].nu[1]});
        }
        hs[b].tab = it->second;
    }
    void *dspecs;
    CIL_TRY(c.cb->alloc(&dspecs, sizeof(TabSpec) * specs.size()));
    CIL_HIP(hipMemcpyAsync(dspecs, specs.data(), sizeof(TabSpec) * specs.size(), hipMemcpyHostToDevice, c.st));
    if (vform) {
        const size_t per = (size_t)2 * 3 * (n / 2 + 1) * n;
        CIL_TRY(c.cb->alloc(tables, sizeof(T) * per * specs.size()));
        dim3 grid((unsigned)((2 * (n / 2 + 1) * n + 255) / 256), (unsigned)specs.size());
        hipLaunchKernelGGL(k_make_vtables<T>, grid, dim3(256), 0, c.st, (const TabSpec *)dspecs, (int)specs.size(), n,
                           dtt, (T *)*tables);
        return check_launch("k_make_vtables");
    }
    CIL_TRY(c.cb->alloc(tables, sizeof(T) * (size_t)2 * n * n * specs.size()));
    dim3 grid((2 * n * n + 255) / 256, (unsigned)specs.size());
    hipLaunchKernelGGL(k_make_tables<T>, grid, dim3(256), 0, c.st, (const TabSpec *)dspecs, (int)specs.size(), n, dtt,
                       (T *)*tables);
    return check_launch("k_make_tables");
}

// Per-solve results of fused launches (steps, last residual, status and, for
// mixed launches, the switch step) back to the host: pinned staging, so the
// copies are queued without blocking, and one wait.
struct HostResults {
    const long long *steps;
    const double *res;
    const int *stat;
    const long long *sw;
};
int fetch_results(SimCtx &c, int B, const long long *dsteps, const double *dres, const int *dstat,
                  const long long *dsw, HostResults *out)
{
    char *hb;
    const size_t b8 = sizeof(long long) * (size_t)B;
    CIL_TRY(host_stage(HS_STEP, 3 * b8 + sizeof(int) * (size_t)B, (void **)&hb));
    out->steps = (const long long *)hb;
    out->res = (const double *)(hb + b8);
    out->sw = dsw ? (const long long *)(hb + 2 * b8) : nullptr;
    out->stat = (const int *)(hb + 3 * b8);
    CIL_HIP(hipMemcpyAsync(hb, dsteps, b8, hipMemcpyDeviceToHost, c.st));
    CIL_HIP(hipMemcpyAsync(hb + b8, dres, b8, hipMemcpyDeviceToHost, c.st));
    CIL_HIP(hipMemcpyAsync(hb + 3 * b8, dstat, sizeof(int) * (size_t)B, hipMemcpyDeviceToHost, c.st));
    if (dsw) CIL_HIP(hipMemcpyAsync(hb + 2 * b8, dsw, b8, hipMemcpyDeviceToHost, c.st));
    return stream_wait(c.st);
}

// Fused solves, all sides in one go: every workgroup runs its solve from
// steps[b] until its stop rule fires.  `dsteps/dres/dstat` are per-solve
// device arrays; the host copies are refreshed after the launches.
template <typename T>
int run_fused(SimCtx &c, const std::map<int, std::vector<int>> &byn, std::vector<DevSolve> &hs, DevSolve *dS, T *state,
              bool quad, double floor_coef, long long *dsteps, double *dres, int *dstat, const MixedArgs *mx = nullptr)
{
    if (byn.empty()) return CIL_OK;
    std::vector<void *> tabs, tabs64;
    std::vector<char> mixed;
    for (auto &kv : byn) {
        void *t, *t64 = nullptr;
        CIL_TRY(make_tables<T>(c, kv.first, kv.second, hs, &t,
                               quad && kQuadShape[quad_shape(std::is_same<T, float>::value, kv.first)].vform));
        const bool mix = mx && mixed_supported(kv.first, quad);
        if (mix && !mx->refine && !g_polish_separate)
            CIL_TRY(make_tables<double>(c, kv.first, kv.second, hs, &t64, kQuadShape[quad_shape(false, kv.first)].vform));
        tabs.push_back(t);
        tabs64.push_back(t64);
        mixed.push_back(mix);
    }
    const int B = (int)hs.size();
    CIL_HIP(hipMemcpyAsync(dS, hs.data(), sizeof(DevSolve) * B, hipMemcpyHostToDevice, c.st));
    std::vector<long long> hsteps(c.steps.begin(), c.steps.end());
    CIL_HIP(hipMemcpyAsync(dsteps, hsteps.data(), sizeof(long long) * B, hipMemcpyHostToDevice, c.st));
    PersistArgs pa{(long long)c.max_steps, c.tol, c.check, floor_coef, dsteps, dres, dstat, g_wave_priority};
    // Several grid sides: each side's persistent kernel on its own stream, the
    // most expensive (n^2 log n x solves) launched first, joined back into the
    // caller's stream, so the call stays ordered on it.
    std::vector<std::pair<double, int>> order;
    {
        int gi = 0;
        for (auto &kv : byn) {
            const double n = kv.first;
            order.push_back({-n * n * std::log2(n) * (double)kv.second.size(), gi++});
        }
        std::sort(order.begin(), order.end());
    }
    std::vector<int *> dls;
    for (auto &kv : byn) {
        int *dl;
        CIL_TRY(c.cb->alloc((void **)&dl, sizeof(int) * kv.second.size()));
        CIL_HIP(hipMemcpyAsync(dl, kv.second.data(), sizeof(int) * kv.second.size(), hipMemcpyHostToDevice, c.st));
        dls.push_back(dl);
    }
    AuxStreams *aux = nullptr;
    const int ng = (int)byn.size();
    if (ng > 1) {
        CIL_TRY(aux_streams(ng, &aux));
        CIL_HIP(hipEventRecord(aux->ev[0], c.st));
    }
    std::vector<const std::pair<const int, std::vector<int>> *> groups;
    for (auto &kv : byn) groups.push_back(&kv);
    for (auto &o : order) {
        const int gi = o.second;
        const auto &kv = *groups[gi];
        hipStream_t gst = c.st;
        if (aux) {
            gst = aux->st[gi];
            CIL_HIP(hipStreamWaitEvent(gst, aux->ev[0], 0));
        }
        const int shape = quad_shape(std::is_same<T, float>::value, kv.first);
        if constexpr (std::is_same<T, float>::value) {
            if (mixed[gi]) {
                PersistArgs pa64 = pa;
                pa64.floor_coef = 0.0;
                // separate polish: the FP32 phase here, the continuation in a
                // launch of its own over the solves at their floor (run_phase2)
                const int mode = g_polish_separate ? 1 : 0;
                const ProfMark pm = prof_begin(kv.first == 32 ? (mode ? "k_fused_q_mixed_n32_phase1" : "k_fused_q_mixed_n32")
                                                              : (mode ? "k_fused_q_mixed_n64_phase1" : "k_fused_q_mixed_n64"),
                                               gst);
                const int rc = launch_quad_mixed(kv.first, (int)kv.second.size(), dS, dls[gi], state, mx->state64,
                                                 (const float *)tabs[gi], (const double *)tabs64[gi], c.model, c.dt,
                                                 pa, pa64, mx->sw, mx->refine, mode, gst);
                prof_end(pm, gst);
                if (rc) return set_error(rc, "no mixed-precision kernel for n = %d", kv.first);
                CIL_TRY(check_launch("k_fused_q_mixed"));
                if (aux) {
                    CIL_HIP(hipEventRecord(aux->ev[1 + gi], gst));
                    CIL_HIP(hipStreamWaitEvent(c.st, aux->ev[1 + gi], 0));
                }
                continue;
            }
        }
        CIL_TRY(launch_persistent<T>(kv.first, quad, shape, (int)kv.second.size(), dS, dls[gi], state,
                                     (const T *)tabs[gi], c.model, c.dt, pa, gst));
        if (aux) {
            CIL_HIP(hipEventRecord(aux->ev[1 + gi], gst));
            CIL_HIP(hipStreamWaitEvent(c.st, aux->ev[1 + gi], 0));
        }
    }
    HostResults h;
    CIL_TRY(fetch_results(c, B, dsteps, dres, dstat, mx ? mx->sw : nullptr, &h));
    for (size_t gi = 0; gi < groups.size(); ++gi)
        for (int b : groups[gi]->second) {
            c.steps[b] = h.steps[b];
            c.fres[b] = h.res[b];
            c.status[b] = h.stat[b];
            if (mixed[gi]) c.sw[b] = h.sw[b];
        }
    return CIL_OK;
}

// The mixed kernel's continuation as a launch of its own (mode 2) over FP32
// solves that its FP32-phase launch (mode 1) left at their floor: FP64 steps,
// or the refinement form with `refine`.  state64: same element layout as
// `state`.
int run_phase2(SimCtx &c, const std::map<int, std::vector<int>> &byn, std::vector<DevSolve> &hs, DevSolve *dS,
               float *state, double *state64, long long *sw, bool refine, long long *dsteps, double *dres, int *dstat)
{
    if (byn.empty()) return CIL_OK;
    const int B = (int)hs.size();
    std::vector<void *> tabs, tabs64;
    for (auto &kv : byn) {
        void *t, *t64 = nullptr;
        CIL_TRY(make_tables<float>(c, kv.first, kv.second, hs, &t, kQuadShape[quad_shape(true, kv.first)].vform));
        if (!refine)
            CIL_TRY(make_tables<double>(c, kv.first, kv.second, hs, &t64, kQuadShape[quad_shape(false, kv.first)].vform));
        tabs.push_back(t);
        tabs64.push_back(t64);
    }
    CIL_HIP(hipMemcpyAsync(dS, hs.data(), sizeof(DevSolve) * B, hipMemcpyHostToDevice, c.st));
    std::vector<long long> hsteps(c.steps.begin(), c.steps.end());
    CIL_HIP(hipMemcpyAsync(dsteps, hsteps.data(), sizeof(long long) * B, hipMemcpyHostToDevice, c.st));
    const PersistArgs pa{(long long)c.max_steps, c.tol, c.check, 0.0, dsteps, dres, dstat, g_wave_priority};
    size_t gi = 0;
    for (auto &kv : byn) {
        int *dl;
        CIL_TRY(c.cb->alloc((void **)&dl, sizeof(int) * kv.second.size()));
        CIL_HIP(hipMemcpyAsync(dl, kv.second.data(), sizeof(int) * kv.second.size(), hipMemcpyHostToDevice, c.st));
        const ProfMark pm =
            prof_begin(kv.first == 32 ? "k_fused_q_mixed_n32_phase2" : "k_fused_q_mixed_n64_phase2", c.st);
        const int rc = launch_quad_mixed(kv.first, (int)kv.second.size(), dS, dl, state, state64,
                                         (const float *)tabs[gi], (const double *)tabs64[gi], c.model, c.dt, pa, pa,
                                         sw, refine, 2, c.st);
        ++gi;
        prof_end(pm, c.st);
        if (rc) return set_error(rc, "no mixed-precision kernel for n = %d", kv.first);
        CIL_TRY(check_launch("k_fused_q_mixed"));
    }
    HostResults h;
    CIL_TRY(fetch_results(c, B, dsteps, dres, dstat, nullptr, &h));
    for (auto &kv : byn)
        for (int b : kv.second) {
            c.steps[b] = h.steps[b];
            c.fres[b] = h.res[b];
            c.status[b] = h.stat[b];
        }
    return CIL_OK;
}

// Second-order fused solves (line variant; n = 32, and n = 64 in FP32, where
// state and history fit the LDS of one workgroup), one launch per grid side,
// in order on the caller's stream.
bool sbdf2_fused_supported(int n, bool f32) { return n == 32 || (n == 64 && f32); }

template <typename T>
int run_fused_sbdf2(SimCtx &c, const std::map<int, std::vector<int>> &byn, std::vector<DevSolve> &hs, DevSolve *dS,
                    T *state, double floor_coef, long long *dsteps, double *dres, int *dstat)
{
    if (byn.empty()) return CIL_OK;
    const bool f32 = std::is_same<T, float>::value;
    std::vector<void *> tabE, tabB;
    for (auto &kv : byn) {
        void *te, *tb;
        CIL_TRY(make_tables<T>(c, kv.first, kv.second, hs, &te, false, c.dt));
        CIL_TRY(make_tables<T>(c, kv.first, kv.second, hs, &tb, false, 2.0 * c.dt / 3.0));
        tabE.push_back(te);
        tabB.push_back(tb);
    }
    const int B = (int)hs.size();
    CIL_HIP(hipMemcpyAsync(dS, hs.data(), sizeof(DevSolve) * B, hipMemcpyHostToDevice, c.st));
    std::vector<long long> hsteps(c.steps.begin(), c.steps.end());
    CIL_HIP(hipMemcpyAsync(dsteps, hsteps.data(), sizeof(long long) * B, hipMemcpyHostToDevice, c.st));
    PersistArgs pa{(long long)c.max_steps, c.tol, c.check, floor_coef, dsteps, dres, dstat, 0.0};
    int gi = 0;
    for (auto &kv : byn) {
        const int n = kv.first, nl = (int)kv.second.size();
        int *dl;
        CIL_TRY(c.cb->alloc((void **)&dl, sizeof(int) * nl));
        CIL_HIP(hipMemcpyAsync(dl, kv.second.data(), sizeof(int) * nl, hipMemcpyHostToDevice, c.st));
        const T *te = (const T *)tabE[gi], *tb = (const T *)tabB[gi];
        ++gi;
        const char *name = n == 32 ? (f32 ? "k_fused_sbdf2_f32_n32" : "k_fused_sbdf2_f64_n32") : "k_fused_sbdf2_f32_n64";
        const ProfMark pm = prof_begin(name, c.st);
        if (n == 32)
            hipLaunchKernelGGL((k_fused_sbdf2<T, 32>), dim3(nl), dim3(64), 0, c.st, dS, dl, state, te, tb, c.model,
                               c.dt, pa);
        else if constexpr (std::is_same<T, float>::value) {
            if (n == 64)
                hipLaunchKernelGGL((k_fused_sbdf2<T, 64>), dim3(nl), dim3(128), 0, c.st, dS, dl, state, te, tb,
                                   c.model, c.dt, pa);
        }
        prof_end(pm, c.st);
        CIL_TRY(check_launch(name));
    }
    HostResults h;
    CIL_TRY(fetch_results(c, B, dsteps, dres, dstat, nullptr, &h));
    for (auto &kv : byn)
        for (int b : kv.second) {
            c.steps[b] = h.steps[b];
            c.fres[b] = h.res[b];
            c.status[b] = h.stat[b];
        }
    return CIL_OK;
}

// Plain solves: host-driven lockstep loop from a common step `start`; a
// launch per stage per step, the residual read back every check_every steps.
template <typename T>
int run_plain(SimCtx &c, std::vector<PlainGroup> &groups, const DevSolve *dS, T *state, int64_t start,
              double floor_coef, StepResults R, int B)
{
    std::vector<unsigned long long> h_resid(B), h_maxabs(B);
    std::vector<int> h_bad(B);
    int64_t step = start;
    auto any_active = [&]() {
        for (auto &g : groups)
            if (!g.active.empty()) return true;
        return false;
    };
    while (step < c.max_steps && any_active()) {
        const int64_t next = std::min<int64_t>(c.max_steps, (step / c.check + 1) * c.check);
        const int K = (int)(next - step);
        for (auto &g : groups) {
            if (g.active.empty()) continue;
            const int nl = (int)g.active.size();
            CIL_HIP(hipMemcpyAsync(g.dlist, g.active.data(), sizeof(int) * nl, hipMemcpyHostToDevice, c.st));
            hipLaunchKernelGGL(k_clear_results, dim3((nl + 255) / 256), dim3(256), 0, c.st, g.dlist, nl, R);
            const Sbdf2Args<T> bdf{(T *)c.uh, (T *)c.fh, step};
            CIL_TRY(launch_plain<T>(g, dS, state, nl, c.model, c.dt, K, R, c.st, c.scheme ? &bdf : nullptr));
        }
        CIL_HIP(hipMemcpyAsync(h_resid.data(), R.resid, sizeof(unsigned long long) * B, hipMemcpyDeviceToHost, c.st));
        CIL_HIP(hipMemcpyAsync(h_maxabs.data(), R.maxabs, sizeof(unsigned long long) * B, hipMemcpyDeviceToHost, c.st));
        CIL_HIP(hipMemcpyAsync(h_bad.data(), R.bad, sizeof(int) * B, hipMemcpyDeviceToHost, c.st));
        CIL_HIP(hipStreamSynchronize(c.st));
        step = next;
        for (auto &g : groups) {
            std::vector<int> keep;
            for (int b : g.active) {
                double dmax, amax;
                std::memcpy(&dmax, &h_resid[b], 8);
                std::memcpy(&amax, &h_maxabs[b], 8);
                const double r = dmax / c.dt;
                c.steps[b] = step;
                if (h_bad[b]) {
                    c.status[b] = CIL_SOLVE_NONFINITE;
                    c.fres[b] = NAN;
                    continue;
                }
                c.fres[b] = r;
                if (c.tol > 0.0 && r < c.tol) {
                    c.status[b] = CIL_SOLVE_OK;
                    continue;
                }
                if (c.tol > 0.0 && floor_coef > 0.0 && r < floor_coef * amax) {
                    c.status[b] = CIL_SOLVE_FP32_FLOOR;
                    continue;
                }
                if (step >= c.max_steps) {
                    c.status[b] = c.tol > 0.0 ? CIL_SOLVE_MAXSTEPS : CIL_SOLVE_OK;
                    continue;
                }
                keep.push_back(b);
            }
            g.active.swap(keep);
        }
    }
    return CIL_OK;
}

template <typename T>
int make_plain_groups(SimCtx &c, const std::map<int, std::vector<int>> &byn, std::vector<PlainGroup> &out)
{
    for (auto &kv : byn) {
        PlainGroup g;
        g.n = kv.first;
        g.active = kv.second;
        g.work_cap = kv.second.size();
        CIL_TRY(c.cb->alloc((void **)&g.dlist, sizeof(int) * g.work_cap));
        CIL_TRY(c.cb->alloc(&g.work, sizeof(T) * (size_t)2 * g.work_cap * 2 * g.n * g.n));
        out.push_back(g);
    }
    return CIL_OK;
}

}  // namespace

int simulate_impl(cil_model model, cil_precision prec, const cil_problem *probs, int B, void *state,
                  const int64_t *offs, const cil_stepping *stp, cil_solve_report *reports, hipStream_t st, int scheme)
{
    const bool f32 = (prec == CIL_FP32);
    const int floor_ulps = stp->fp32_floor_ulps > 0 ? stp->fp32_floor_ulps : 8;
    CallBuffers cb;
    SimCtx c;
    c.model = (int)model;
    c.dt = stp->dt;
    c.tol = stp->tol;
    c.max_steps = stp->max_steps;
    c.check = stp->check_every;
    c.floor_coef32 = (f32 && stp->tol > 0.0) ? floor_ulps * std::ldexp(1.0, -24) / stp->dt : 0.0;
    c.st = st;
    c.cb = &cb;
    c.steps.assign(B, 0);
    c.fres.assign(B, 0.0);
    c.status.assign(B, CIL_SOLVE_OK);
    const bool polish = f32 && stp->polish && stp->tol > 0.0;
    c.polish = polish ? stp->polish : 0;
    const bool quad = stp->path != CIL_PATH_FUSED_LINE;
    if (scheme) {
        if (stp->path == CIL_PATH_FUSED_QUAD)
            return set_error(CIL_EUNSUPPORTED, "the second-order stepper has no quad-lane kernel");
        if (polish)
            return set_error(CIL_EUNSUPPORTED, "the second-order stepper has no FP64 polish: set polish = 0");
    }
    c.scheme = scheme;

    std::vector<DevSolve> hs(B);
    std::vector<int64_t> elems(B);
    int64_t total = 0;
    for (int b = 0; b < B; ++b) {
        const cil_problem &pr = probs[b];
        DevSolve d{};
        d.n = pr.n;
        d.off = offs ? offs[b] : total;
        const double h = pr.L / (double)(pr.n - 1);
        d.inv_h2 = 1.0 / (h * h);
        d.nu[0] = pr.nu[0];
        d.nu[1] = pr.nu[1];
        for (int k = 0; k < 4; ++k) d.p[k] = pr.p[k];
        hs[b] = d;
        elems[b] = 2ll * pr.n * pr.n;
        total += elems[b];
    }

    // phase 1: fused sides run persistently, the rest in the plain lockstep loop
    std::map<int, std::vector<int>> fused_byn, plain_byn;
    for (int b = 0; b < B; ++b) {
        const int n = hs[b].n;
        const bool fs = scheme ? sbdf2_fused_supported(n, f32) : fused_supported(n, f32);
        if (stp->path >= CIL_PATH_FUSED && !fs)
            return set_error(CIL_EUNSUPPORTED, "no fused %sstepper for n = %d in %s", scheme ? "second-order " : "", n,
                             f32 ? "FP32" : "FP64");
        if (fs && stp->path != CIL_PATH_PLAIN) fused_byn[n].push_back(b);
        else plain_byn[n].push_back(b);
    }
    if (scheme && !plain_byn.empty()) {              // the plain back-end keeps the history in HBM
        int64_t end = 0;
        for (int b = 0; b < B; ++b) end = std::max<int64_t>(end, hs[b].off + elems[b]);
        const size_t es = f32 ? sizeof(float) : sizeof(double);
        CIL_TRY(cb.alloc(&c.uh, es * (size_t)end));
        CIL_TRY(cb.alloc(&c.fh, es * (size_t)end));
    }
    DevSolve *dS;
    long long *dsteps;
    double *dres;
    int *dstat;
    CIL_TRY(cb.alloc((void **)&dS, sizeof(DevSolve) * B));
    CIL_TRY(cb.alloc((void **)&dsteps, sizeof(long long) * B));
    CIL_TRY(cb.alloc((void **)&dres, sizeof(double) * B));
    CIL_TRY(cb.alloc((void **)&dstat, sizeof(int) * B));
    CIL_TRY(fill_zero(dstat, sizeof(int) * B, st));
    StepResults R;
    CIL_TRY(cb.alloc((void **)&R.resid, sizeof(unsigned long long) * B));
    CIL_TRY(cb.alloc((void **)&R.maxabs, sizeof(unsigned long long) * B));
    CIL_TRY(cb.alloc((void **)&R.bad, sizeof(int) * B));

    c.sw.assign(B, -1);
    MixedArgs mx{nullptr, nullptr, c.polish == 2};
    bool use_mixed = false;
    if (polish)
        for (auto &kv : fused_byn) use_mixed |= mixed_supported(kv.first, quad);
    if (use_mixed) {
        int64_t end = 0;
        for (int b = 0; b < B; ++b) end = std::max<int64_t>(end, hs[b].off + elems[b]);
        CIL_TRY(cb.alloc((void **)&mx.state64, sizeof(double) * (size_t)end));
        CIL_TRY(cb.alloc((void **)&mx.sw, sizeof(long long) * B));
    }
    if (scheme) {
        if (f32) CIL_TRY(run_fused_sbdf2<float>(c, fused_byn, hs, dS, (float *)state, c.floor_coef32, dsteps, dres, dstat));
        else CIL_TRY(run_fused_sbdf2<double>(c, fused_byn, hs, dS, (double *)state, 0.0, dsteps, dres, dstat));
    } else if (f32) {
        CIL_TRY(run_fused<float>(c, fused_byn, hs, dS, (float *)state, quad, c.floor_coef32, dsteps, dres, dstat,
                                 use_mixed ? &mx : nullptr));
    } else {
        CIL_TRY(run_fused<double>(c, fused_byn, hs, dS, (double *)state, quad, 0.0, dsteps, dres, dstat));
    }
    if (!plain_byn.empty()) {
        CIL_HIP(hipMemcpyAsync(dS, hs.data(), sizeof(DevSolve) * B, hipMemcpyHostToDevice, st));
        std::vector<PlainGroup> pg;
        if (f32) {
            CIL_TRY(make_plain_groups<float>(c, plain_byn, pg));
            CIL_TRY(run_plain<float>(c, pg, dS, (float *)state, 0, c.floor_coef32, R, B));
        } else {
            CIL_TRY(make_plain_groups<double>(c, plain_byn, pg));
            CIL_TRY(run_plain<double>(c, pg, dS, (double *)state, 0, 0.0, R, B));
        }
    }

    // phase 2: FP32 solves stopped at the FP32 floor continue: those whose
    // FP32 phase ran in the mixed kernel (separate polish) in its second
    // launch, the others in FP64 steps
    std::vector<int64_t> steps64(B, 0);
    std::vector<int> promoted;
    std::map<int, std::vector<int>> cont_byn;
    for (int b = 0; b < B; ++b) {
        if (c.sw[b] >= 0) steps64[b] = c.steps[b] - c.sw[b];     // polished inside the mixed launch
        if (!polish || c.status[b] != CIL_SOLVE_FP32_FLOOR) continue;
        if (c.sw[b] >= 0) cont_byn[hs[b].n].push_back(b);
        else promoted.push_back(b);
    }
    if (!cont_byn.empty()) {
        for (auto &kv : cont_byn)
            for (int b : kv.second) c.status[b] = CIL_SOLVE_OK;
        CIL_TRY(run_phase2(c, cont_byn, hs, dS, (float *)state, mx.state64, mx.sw, c.polish == 2, dsteps, dres,
                           dstat));
        for (auto &kv : cont_byn)
            for (int b : kv.second) steps64[b] = c.steps[b] - c.sw[b];
    }
    if (!promoted.empty()) {
        std::vector<DevSolve> hs64 = hs;
        int64_t t = 0;
        for (int b = 0; b < B; ++b) {
            hs64[b].off = t;
            t += elems[b];
        }
        double *state64;
        DevSolve *dS64;
        int *dprom;
        CIL_TRY(cb.alloc((void **)&state64, sizeof(double) * std::max<int64_t>(t, 1)));
        CIL_TRY(cb.alloc((void **)&dS64, sizeof(DevSolve) * B));
        CIL_TRY(cb.alloc((void **)&dprom, sizeof(int) * promoted.size()));
        CIL_HIP(hipMemcpyAsync(dS, hs.data(), sizeof(DevSolve) * B, hipMemcpyHostToDevice, st));
        CIL_HIP(hipMemcpyAsync(dS64, hs64.data(), sizeof(DevSolve) * B, hipMemcpyHostToDevice, st));
        CIL_HIP(hipMemcpyAsync(dprom, promoted.data(), sizeof(int) * promoted.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL((k_convert_solves<float, double>), dim3(16, (unsigned)promoted.size()), dim3(256), 0, st,
                           (const DevSolve *)dS, (const DevSolve *)dS64, dprom, (const float *)state, state64);
        CIL_TRY(check_launch("k_convert_solves"));
        std::vector<int64_t> before(B);
        for (int b = 0; b < B; ++b) before[b] = c.steps[b];
        std::map<int, std::vector<int>> fz;                            // n -> solves (fused FP64)
        std::map<std::pair<int, int64_t>, std::vector<int>> pz;        // (n, start) -> solves (plain FP64)
        for (int b : promoted) {
            c.status[b] = CIL_SOLVE_OK;
            if (fused_supported(hs[b].n, false) && stp->path != CIL_PATH_PLAIN) fz[hs[b].n].push_back(b);
            else pz[std::make_pair(hs[b].n, c.steps[b])].push_back(b);
        }
        CIL_TRY(run_fused<double>(c, fz, hs64, dS64, state64, quad, 0.0, dsteps, dres, dstat));
        if (!pz.empty()) CIL_HIP(hipMemcpyAsync(dS64, hs64.data(), sizeof(DevSolve) * B, hipMemcpyHostToDevice, st));
        for (auto &kv : pz) {
            std::map<int, std::vector<int>> one;
            one[kv.first.first] = kv.second;
            std::vector<PlainGroup> pg;
            CIL_TRY(make_plain_groups<double>(c, one, pg));
            CIL_TRY(run_plain<double>(c, pg, dS64, state64, kv.first.second, 0.0, R, B));
        }
        for (int b : promoted) steps64[b] = c.steps[b] - before[b];
        hipLaunchKernelGGL((k_convert_solves<double, float>), dim3(16, (unsigned)promoted.size()), dim3(256), 0, st,
                           (const DevSolve *)dS64, (const DevSolve *)dS, dprom, (const double *)state64, (float *)state);
        CIL_TRY(check_launch("k_convert_solves"));
    }
    CIL_TRY(stream_wait(st));
    cb.done = true;

    int rc = CIL_OK;
    for (int b = 0; b < B; ++b) {
        if (c.status[b] == CIL_SOLVE_NONFINITE) rc = CIL_ENONFINITE;
        if (reports) {
            reports[b].steps_taken = c.steps[b];
            reports[b].steps_fp64 = f32 ? steps64[b] : 0;
            reports[b].final_resid = c.fres[b];
            reports[b].status = c.status[b];
            reports[b].reserved = 0;
        }
    }
    if (rc == CIL_ENONFINITE) set_error(rc, "a solve produced a non-finite value");
    return rc;
}

// ------------------------------------------------------------------ plans
// A simulate plan binds one batch of fused solves (problems, layout,
// stepping, the state buffer) to device-resident spectral tables, solve
// descriptors and per-solve result arrays, and to one instantiated HIP graph:
// a clear of the results, then one persistent kernel per grid side, forked
// over plan-owned streams (default priority) and joined.  Each launch replays
// the graph: every solve starts at step 0 from what the state holds.
struct SimPlan {
    struct Group {
        int n = 0;
        std::vector<int> ids;
        int shape = 0;
        void *tab[2] = {nullptr, nullptr};    // X-form, V-form divisor tables
        int *dl = nullptr;
        double tuned_ms[kQuadShapes] = {};
    };
    int dev = 0;
    int model = 0;
    bool f32 = false, quad = true;
    double dt = 0.0;
    PersistArgs pa{};
    void *state = nullptr;
    size_t state_bytes = 0;
    int B = 0;
    std::vector<DevSolve> hs;
    std::vector<Group> groups;            // launch order: most expensive first
    CallBuffers bufs;
    DevSolve *dS = nullptr;
    std::vector<hipStream_t> st;          // st[0] captures; st[g] runs group g
    std::vector<hipEvent_t> ev;           // ev[0] fork, ev[g] join of group g
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~SimPlan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipStream_t s : st) (void)hipStreamDestroy(s);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

namespace {

// tables of group g for the divisor form of `shape` (built once per form)
int plan_tables(SimPlan &p, SimPlan::Group &g, int shape, hipStream_t st)
{
    const int vf = (p.quad && kQuadShape[shape].vform) ? 1 : 0;
    if (g.tab[vf]) return CIL_OK;
    SimCtx c;
    c.model = p.model;
    c.dt = p.dt;
    c.st = st;
    c.cb = &p.bufs;
    if (p.f32) CIL_TRY(make_tables<float>(c, g.n, g.ids, p.hs, &g.tab[vf], vf != 0));
    else CIL_TRY(make_tables<double>(c, g.n, g.ids, p.hs, &g.tab[vf], vf != 0));
    // the table index of each solve depends only on (h, nu) order within the
    // group, the same for both forms; descriptors are re-sent after a build
    CIL_HIP(hipMemcpyAsync(p.dS, p.hs.data(), sizeof(DevSolve) * p.B, hipMemcpyHostToDevice, st));
    return CIL_OK;
}

int plan_launch_group(SimPlan &p, SimPlan::Group &g, int shape, void *state, const PersistArgs &pa, hipStream_t st)
{
    const int vf = (p.quad && kQuadShape[shape].vform) ? 1 : 0;
    if (p.f32)
        return launch_persistent<float>(g.n, p.quad, shape, (int)g.ids.size(), p.dS, g.dl, (float *)state,
                                        (const float *)g.tab[vf], p.model, p.dt, pa, st);
    return launch_persistent<double>(g.n, p.quad, shape, (int)g.ids.size(), p.dS, g.dl, (double *)state,
                                     (const double *)g.tab[vf], p.model, p.dt, pa, st);
}

// the graph's work, enqueued on the capturing stream p.st[0]
int plan_enqueue(SimPlan &p)
{
    hipStream_t cs = p.st[0];
    CIL_TRY(fill_zero(p.pa.steps, sizeof(long long) * p.B, cs));
    CIL_TRY(fill_zero(p.pa.resid, sizeof(double) * p.B, cs));
    CIL_TRY(fill_zero(p.pa.status, sizeof(int) * p.B, cs));
    const int ng = (int)p.groups.size();
    if (ng > 1) CIL_HIP(hipEventRecord(p.ev[0], cs));
    for (int g = 1; g < ng; ++g) CIL_HIP(hipStreamWaitEvent(p.st[g], p.ev[0], 0));
    for (int g = 0; g < ng; ++g) CIL_TRY(plan_launch_group(p, p.groups[g], p.groups[g].shape, p.state, p.pa, p.st[g]));
    for (int g = 1; g < ng; ++g) {
        CIL_HIP(hipEventRecord(p.ev[g], p.st[g]));
        CIL_HIP(hipStreamWaitEvent(cs, p.ev[g], 0));
    }
    return CIL_OK;
}

int plan_build_graph(SimPlan &p)
{
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    p.exec = nullptr;
    p.graph = nullptr;
    CIL_HIP(hipStreamBeginCapture(p.st[0], hipStreamCaptureModeThreadLocal));
    const int rc = plan_enqueue(p);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p.st[0], &g);
    if (rc != CIL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_error(CIL_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    p.graph = g;
    CIL_HIP(hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0));
    return CIL_OK;
}

}  // namespace

int plan_create(cil_model model, cil_precision prec, const cil_problem *probs, int B, void *state, const int64_t *offs,
                const cil_stepping *stp, hipStream_t st, SimPlan **out)
{
    const bool f32 = (prec == CIL_FP32);
    if (stp->path == CIL_PATH_PLAIN) return set_error(CIL_EUNSUPPORTED, "plans run the fused steppers only");
    if (f32 && stp->polish && stp->tol > 0.0)
        return set_error(CIL_EINVAL, "plans do not polish in FP64: set polish = 0 (FP32 floor is then a status)");
    std::unique_ptr<SimPlan> p(new SimPlan());
    CIL_TRY(current_device(&p->dev));
    p->model = (int)model;
    p->f32 = f32;
    p->quad = stp->path != CIL_PATH_FUSED_LINE;
    p->dt = stp->dt;
    p->state = state;
    p->B = B;
    p->hs.resize(B);
    int64_t total = 0, end = 0;
    std::map<int, std::vector<int>> byn;
    for (int b = 0; b < B; ++b) {
        const cil_problem &pr = probs[b];
        if (!fused_supported(pr.n, f32))
            return set_error(CIL_EUNSUPPORTED, "no fused stepper for n = %d in %s", pr.n, f32 ? "FP32" : "FP64");
        DevSolve d{};
        d.n = pr.n;
        d.off = offs ? offs[b] : total;
        const double h = pr.L / (double)(pr.n - 1);
        d.inv_h2 = 1.0 / (h * h);
        d.nu[0] = pr.nu[0];
        d.nu[1] = pr.nu[1];
        for (int k = 0; k < 4; ++k) d.p[k] = pr.p[k];
        p->hs[b] = d;
        total += 2ll * pr.n * pr.n;
        end = std::max<int64_t>(end, d.off + 2ll * pr.n * pr.n);
        byn[pr.n].push_back(b);
    }
    p->state_bytes = (size_t)end * (f32 ? 4 : 8);
    std::vector<std::pair<double, int>> order;
    for (auto &kv : byn) order.push_back({-(double)kv.first * kv.first * std::log2((double)kv.first) * kv.second.size(),
                                          kv.first});
    std::sort(order.begin(), order.end());
    CIL_TRY(p->bufs.alloc((void **)&p->dS, sizeof(DevSolve) * B));
    long long *dsteps;
    double *dres;
    int *dstat;
    CIL_TRY(p->bufs.alloc((void **)&dsteps, sizeof(long long) * B));
    CIL_TRY(p->bufs.alloc((void **)&dres, sizeof(double) * B));
    CIL_TRY(p->bufs.alloc((void **)&dstat, sizeof(int) * B));
    const double floor_coef =
        (f32 && stp->tol > 0.0) ? (stp->fp32_floor_ulps > 0 ? stp->fp32_floor_ulps : 8) * std::ldexp(1.0, -24) / stp->dt
                                : 0.0;
    p->pa = PersistArgs{(long long)stp->max_steps, stp->tol, stp->check_every, floor_coef, dsteps, dres, dstat,
                        g_wave_priority};
    CIL_HIP(hipMemcpyAsync(p->dS, p->hs.data(), sizeof(DevSolve) * B, hipMemcpyHostToDevice, st));
    for (auto &o : order) {
        SimPlan::Group g;
        g.n = o.second;
        g.ids = byn[g.n];
        g.shape = p->quad ? quad_shape(f32, g.n) : 0;
        CIL_TRY(p->bufs.alloc((void **)&g.dl, sizeof(int) * g.ids.size()));
        CIL_HIP(hipMemcpyAsync(g.dl, g.ids.data(), sizeof(int) * g.ids.size(), hipMemcpyHostToDevice, st));
        p->groups.push_back(g);
    }
    for (auto &g : p->groups) CIL_TRY(plan_tables(*p, g, g.shape, st));
    const int ng = (int)p->groups.size();
    for (int g = 0; g < std::max(ng, 1); ++g) {
        hipStream_t s;
        CIL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        p->st.push_back(s);
        hipEvent_t e;
        CIL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p->ev.push_back(e);
    }
    CIL_HIP(hipStreamSynchronize(st));     // uploads done before capture and before host vectors go
    CIL_TRY(plan_build_graph(*p));
    *out = p.release();
    return CIL_OK;
}

int plan_tune(SimPlan *p, int64_t steps, hipStream_t st)
{
    if (!p->quad) return set_error(CIL_EINVAL, "tuning chooses among the quad-lane shapes (path is FUSED_LINE)");
    if (steps < 0) return set_error(CIL_EINVAL, "tuning needs steps >= 0");
    CIL_HIP(hipSetDevice(p->dev));
    CallBuffers tb;
    void *scratch;
    long long *tsteps;
    double *tres;
    int *tstat;
    CIL_TRY(tb.alloc(&scratch, p->state_bytes));
    CIL_TRY(tb.alloc((void **)&tsteps, sizeof(long long) * p->B));
    CIL_TRY(tb.alloc((void **)&tres, sizeof(double) * p->B));
    CIL_TRY(tb.alloc((void **)&tstat, sizeof(int) * p->B));
    // steps > 0: fixed-length trials (no stop rule); 0: the plan's own stepping
    const PersistArgs pa = steps > 0 ? PersistArgs{(long long)steps, 0.0, (int)std::min<int64_t>(steps, 1 << 30), 0.0,
                                                   tsteps, tres, tstat}
                                     : PersistArgs{p->pa.max_steps, p->pa.tol, p->pa.check, p->pa.floor_coef, tsteps,
                                                   tres, tstat, p->pa.prio};
    hipEvent_t a, b;
    CIL_HIP(hipEventCreate(&a));
    CIL_HIP(hipEventCreate(&b));
    int rc = CIL_OK;
    for (auto &g : p->groups) {
        int best = -1;
        for (int s = 0; s < kQuadShapes && rc == CIL_OK; ++s) {
            rc = plan_tables(*p, g, s, st);
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && rc == CIL_OK; ++rep) {
                // every trial starts from the same states (a copy of the bound state)
                if (hipMemcpyAsync(scratch, p->state, p->state_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                    (rc = fill_zero(tsteps, sizeof(long long) * p->B, st)) != CIL_OK ||
                    hipEventRecord(a, st) != hipSuccess) {
                    if (rc == CIL_OK) rc = set_error(CIL_EDEVICE, "tuning copy failed");
                    break;
                }
                rc = plan_launch_group(*p, g, s, scratch, pa, st);
                if (rc == CIL_OK && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                                     hipEventElapsedTime(&ms, a, b) != hipSuccess))
                    rc = set_error(CIL_EDEVICE, "tuning timing failed");
            }
            if (rc != CIL_OK) break;
            g.tuned_ms[s] = ms;
            if (best < 0 || ms < g.tuned_ms[best]) best = s;
        }
        if (rc != CIL_OK) break;
        g.shape = best;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    CIL_TRY(rc);
    CIL_HIP(hipStreamSynchronize(st));
    tb.done = true;
    return plan_build_graph(*p);
}

int plan_launch(SimPlan *p, hipStream_t st)
{
    const ProfMark pm = prof_begin("sim_plan_graph", st);
    CIL_HIP(hipGraphLaunch(p->exec, st));
    prof_end(pm, st);
    return CIL_OK;
}

int plan_report(SimPlan *p, cil_solve_report *reports, hipStream_t st)
{
    const int B = p->B;
    std::vector<long long> hsteps(B);
    std::vector<double> hres(B);
    std::vector<int> hstat(B);
    CIL_HIP(hipMemcpyAsync(hsteps.data(), p->pa.steps, sizeof(long long) * B, hipMemcpyDeviceToHost, st));
    CIL_HIP(hipMemcpyAsync(hres.data(), p->pa.resid, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    CIL_HIP(hipMemcpyAsync(hstat.data(), p->pa.status, sizeof(int) * B, hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    int rc = CIL_OK;
    for (int b = 0; b < B; ++b) {
        if (hstat[b] == CIL_SOLVE_NONFINITE) rc = CIL_ENONFINITE;
        if (reports) reports[b] = cil_solve_report{hsteps[b], 0, hres[b], hstat[b], 0};
    }
    if (rc == CIL_ENONFINITE) set_error(rc, "a solve produced a non-finite value");
    return rc;
}

int plan_groups(const SimPlan *p) { return (int)p->groups.size(); }

int plan_group_info(const SimPlan *p, int g, int *n, int *count, int *shape, double *tuned_ms)
{
    if (g < 0 || g >= (int)p->groups.size()) return set_error(CIL_EINVAL, "group %d out of range", g);
    const SimPlan::Group &G = p->groups[g];
    if (n) *n = G.n;
    if (count) *count = (int)G.ids.size();
    if (shape) *shape = G.shape;
    if (tuned_ms)
        for (int s = 0; s < kQuadShapes; ++s) tuned_ms[s] = G.tuned_ms[s];
    return CIL_OK;
}

void plan_destroy(SimPlan *p)
{
    if (!p) return;
    (void)hipSetDevice(p->dev);
    (void)hipDeviceSynchronize();
    p->bufs.done = true;
    delete p;
}

}  // namespace cil
