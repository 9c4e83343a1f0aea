// Pair distances, radius bins and correlation sums (Sec. 2.1, eqs. eCDF and
// CIL) on gfx950.
//
// Canonical squared distance of two patterns a, b of length d:
//   d_k = fl64(a_k - b_k)  (inputs converted to double),
//   D   = RN64(sum_k d_k^2)   -- the exact sum, rounded once.
// Counting rule: a pair lies under radius R_m when D < fl(R_m * R_m).
//
// Fast pass (this file, k_dist_tile): D~ = sum_k d_k^2 in FP64, one pair per
// accumulator, summed sequentially with FMA.  All terms are non-negative, so
// |D~ - sum| <= gamma_d * D~ with gamma_d = d u / (1 - d u), u = 2^-53; with
// the final rounding and a margin, |D~ - D| <= eps_rel * D~, eps_rel =
// (d + 4) 2^-53 * 1.01.  A pair whose D~ is within that band of any
// threshold is recomputed canonically (k_canonical), all others are binned
// from D~ directly: every count is exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cil_internal.hpp"

// The error-free transformations below (two-sum, exact squares split by an
// FMA) are only exact if no product is fused into a later sum: contraction
// off for this file; the fused multiply-adds that are wanted are explicit.
#pragma clang fp contract(off)

namespace cil {

constexpr int TILE = 64;       // pairs per tile side
constexpr int KC = 16;         // k-chunk staged in LDS
constexpr int MAX_M = 255;

struct BinOut {
    const double *thr;          // device [M]: fl(R_m^2), strictly decreasing
    int M;
    double eps_rel;             // band half-width relative to max(D~, thr)
    unsigned long long *hist;   // device [M+1]: pairs per bin value (binned pairs only)
    uint8_t *bins;              // device [nA][nB] or null
    int2 *recheck;              // device list of pairs to recompute
    unsigned long long *nrecheck;
    long long recheck_cap;
    double *dmat;               // device [nA][nB] of D~ or null (range mode)
    int exclude_diag;
    unsigned long long *dmin_bits, *dmax_bits;   // range mode (non-negative doubles)
};

__device__ __forceinline__ double ld(const double *p) { return *p; }
__device__ __forceinline__ double ld(const float *p) { return (double)*p; }

// One 64 x 64 tile of pairs per block of 256 threads; thread (ty, tx) owns
// rows ty + 16 i and columns tx + 16 j, i, j < 4.
template <typename T, bool RANGE>
__global__ __launch_bounds__(256) void k_dist_tile(const T *A, long long nA, const T *B, long long nB,
                                                   long long dim, BinOut o)
{
    __shared__ double sA[TILE][KC + 1];
    __shared__ double sB[TILE][KC + 1];
    __shared__ unsigned int hist[MAX_M + 1];
    __shared__ double sthr[MAX_M];

    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const long long i0 = (long long)blockIdx.y * TILE, j0 = (long long)blockIdx.x * TILE;
    if (!RANGE) {
        for (int m = tid; m <= o.M; m += 256) hist[m] = 0;
        for (int m = tid; m < o.M; m += 256) sthr[m] = o.thr[m];
    }
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

    for (long long k0 = 0; k0 < dim; k0 += KC) {
        __syncthreads();
        for (int e = tid; e < TILE * KC; e += 256) {
            const int r = e / KC, kk = e % KC;
            const long long k = k0 + kk;
            const long long ia = i0 + r, jb = j0 + r;
            sA[r][kk] = (ia < nA && k < dim) ? ld(A + ia * dim + k) : 0.0;
            sB[r][kk] = (jb < nB && k < dim) ? ld(B + jb * dim + k) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sA[ty + 16 * i][kk];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sB[tx + 16 * j][kk];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double dlt = a[i] - b[j];
                    acc[i][j] = fma(dlt, dlt, acc[i][j]);
                }
        }
    }
    __syncthreads();

    if (RANGE) {
        double mn = INFINITY, mx = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long long ia = i0 + ty + 16 * i, jb = j0 + tx + 16 * j;
                if (ia >= nA || jb >= nB) continue;
                if (o.exclude_diag && ia == jb) continue;
                const double D = acc[i][j];
                o.dmat[ia * nB + jb] = D;
                mn = fmin(mn, D);
                mx = fmax(mx, D);
            }
        if (mn < INFINITY) atomicMin(o.dmin_bits, (unsigned long long)__double_as_longlong(mn));
        atomicMax(o.dmax_bits, (unsigned long long)__double_as_longlong(mx));
        return;
    }

#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long ia = i0 + ty + 16 * i, jb = j0 + tx + 16 * j;
            if (ia >= nA || jb >= nB) continue;
            const double D = acc[i][j];
            int bin = 0;
            bool amb = false;
            for (int m = 0; m < o.M; ++m) {
                const double t = sthr[m];
                if (fabs(D - t) <= o.eps_rel * fmax(D, t)) amb = true;
                bin += (D < t);
            }
            if (!isfinite(D)) amb = true;
            if (amb) {
                const unsigned long long slot = atomicAdd(o.nrecheck, 1ull);
                if ((long long)slot < o.recheck_cap) o.recheck[slot] = make_int2((int)ia, (int)jb);
            } else {
                atomicAdd(&hist[bin], 1u);
                if (o.bins) o.bins[ia * nB + jb] = (uint8_t)bin;
            }
        }
    __syncthreads();
    for (int m = tid; m <= o.M; m += 256)
        if (hist[m]) atomicAdd(&o.hist[m], (unsigned long long)hist[m]);
}

// ---------------------------------------------------------------- canonical
// Double-double accumulation of the exact squares, one wavefront per pair,
// then a certified rounding: with the accumulated value S = hi + lo and its
// relative error bound delta, RN(sum) = RN(hi + lo) whenever the interval
// [S - delta S, S + delta S] holds no rounding boundary.  Otherwise (or when
// forced) lane 0 recomputes the sum exactly in a non-overlapping expansion
// (Shewchuk's exact summation) and rounds it once, half to even.

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void dd_add(double &hi, double &lo, double bh, double bl)
{
    double s, e;
    two_sum(hi, bh, s, e);
    e += lo + bl;
    hi = s + e;
    lo = e - (hi - s);
}

template <typename T>
__device__ double exact_d2_serial(const T *a, const T *b, long long dim)
{
    double part[96];
    int np = 0;
    auto add = [&](double x) {
        int k = 0;
        for (int i = 0; i < np; ++i) {
            double y = part[i];
            if (fabs(x) < fabs(y)) {
                const double t = x;
                x = y;
                y = t;
            }
            const double hi = x + y;
            const double lo = y - (hi - x);
            if (lo != 0.0) part[k++] = lo;
            x = hi;
        }
        part[k++] = x;
        np = k;
    };
    for (long long k = 0; k < dim; ++k) {
        const double d = ld(a + k) - ld(b + k);
        const double p = d * d;
        const double e = fma(d, d, -p);
        add(p);
        if (e != 0.0) add(e);
    }
    if (np == 0) return 0.0;
    int m = np;
    double hi = part[--m], lo = 0.0;
    while (m > 0) {
        const double x = hi, y = part[--m];
        hi = x + y;
        lo = y - (hi - x);
        if (lo != 0.0) break;
    }
    if (m > 0 && ((lo < 0.0 && part[m - 1] < 0.0) || (lo > 0.0 && part[m - 1] > 0.0))) {
        const double y = lo * 2.0, x = hi + y;
        if (y == x - hi) hi = x;
    }
    return hi;
}

struct CanonOut {
    // pair source: either an int2 list (recheck) or two index arrays
    const int2 *pairs;
    const unsigned long long *npairs_dev;   // count for the list (clamped to cap)
    long long cap;
    const long long *ia, *jb;
    long long npairs;
    long long nA;               // index bounds for the ia/jb source
    int *bad;                   // set when an ia/jb index is out of range
    // sinks
    double *d2;                 // per pair, or null
    const double *thr;
    int M;
    unsigned long long *hist;   // or null
    uint8_t *bins;              // or null
    long long nB;
    unsigned long long *nexact;
    int force_exact;
};

template <typename T>
__global__ __launch_bounds__(256) void k_canonical(const T *A, const T *B, long long dim, CanonOut o)
{
    const int lane = threadIdx.x & 63;
    const long long w = (long long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const long long np = o.pairs ? (long long)min((unsigned long long)o.cap, *o.npairs_dev) : o.npairs;
    if (w >= np) return;
    long long i, j;
    if (o.pairs) {
        i = o.pairs[w].x;
        j = o.pairs[w].y;
    } else {
        i = o.ia[w];
        j = o.jb[w];
        if (i < 0 || i >= o.nA || j < 0 || j >= o.nB) {
            if (lane == 0) {
                if (o.d2) o.d2[w] = NAN;
                atomicOr(o.bad, 1);
            }
            return;
        }
    }
    const T *a = A + i * dim;
    const T *b = B + j * dim;
    double hi = 0.0, lo = 0.0;
    for (long long k = lane; k < dim; k += 64) {
        const double d = ld(a + k) - ld(b + k);
        const double p = d * d;
        dd_add(hi, lo, p, fma(d, d, -p));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double oh = __shfl_xor(hi, off, 64), ol = __shfl_xor(lo, off, 64);
        dd_add(hi, lo, oh, ol);
    }
    double D;
    if (lane == 0) {
        double R, e;
        two_sum(hi, lo, R, e);
        const double delta = (double)(dim + 64) * 0x1p-100;   // relative error bound
        int ex;
        (void)frexp(R, &ex);                                 // R in [2^(ex-1), 2^ex)
        const double half = ldexp(1.0, ex - 1 - 54);         // smallest half-spacing near R
        const bool certain = isfinite(R) && (fabs(e) + delta * R < half || R == 0.0);
        D = R;
        if (!certain || o.force_exact) {
            D = exact_d2_serial(a, b, dim);
            atomicAdd(o.nexact, 1ull);
        }
        if (o.d2) o.d2[w] = D;
        if (o.hist) {
            int bin = 0;
            for (int m = 0; m < o.M; ++m) bin += (D < o.thr[m]);
            atomicAdd(&o.hist[bin], 1ull);
            if (o.bins) o.bins[i * o.nB + j] = (uint8_t)bin;
        }
    }
}

// ---------------------------------------------------------------- range fix
// Candidates for the canonical extremes: pairs whose D~ lies within the band
// of the fast-pass minimum or maximum.
__global__ void k_range_candidates(const double *dmat, long long nA, long long nB, double lo_thr,
                                   double hi_thr, int exclude_diag, int2 *out,
                                   unsigned long long *count, long long cap)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nA * nB) return;
    const long long i = e / nB, j = e % nB;
    if (exclude_diag && i == j) return;
    const double D = dmat[e];
    if (D <= lo_thr || D >= hi_thr || !isfinite(D)) {
        const unsigned long long s = atomicAdd(count, 1ull);
        if ((long long)s < cap) out[s] = make_int2((int)i, (int)j);
    }
}

// ======================================================================
// Host side.

namespace {
thread_local long long t_pairs = 0, t_rechecked = 0, t_exact = 0;
int g_force_exact = 0;

struct DistScratch {
    double *thr = nullptr;
    unsigned long long *hist = nullptr;
    unsigned long long *nrecheck = nullptr;
    unsigned long long *nexact = nullptr;
    unsigned long long *minmax = nullptr;
    int2 *recheck = nullptr;
    long long cap = 0;
};

int scratch(long long npairs_cap, DistScratch *s)
{
    void *p;
    CIL_TRY(ws_get(WS_DIST_MISC, 4096 + sizeof(double) * 512, &p));
    char *c = (char *)p;
    s->thr = (double *)c;                                   // 256 doubles
    s->hist = (unsigned long long *)(c + 2048);             // 256 counters
    s->nrecheck = (unsigned long long *)(c + 4096);
    s->nexact = s->nrecheck + 1;
    s->minmax = s->nrecheck + 2;
    CIL_TRY(ws_get(WS_DIST_RECHECK, sizeof(int2) * (size_t)std::max<long long>(npairs_cap, 1), &p));
    s->recheck = (int2 *)p;
    s->cap = npairs_cap;
    return CIL_OK;
}

dim3 tile_grid(long long nA, long long nB)
{
    return dim3((unsigned)((nB + TILE - 1) / TILE), (unsigned)((nA + TILE - 1) / TILE));
}

template <typename T>
int run_canonical(const T *A, const T *B, long long dim, CanonOut &co, long long nwaves, hipStream_t st)
{
    if (nwaves <= 0) return CIL_OK;
    const long long blocks = (nwaves + 3) / 4;
    const ProfMark pm = prof_begin("k_canonical", st);
    hipLaunchKernelGGL(k_canonical<T>, dim3((unsigned)blocks), dim3(256), 0, st, A, B, dim, co);
    prof_end(pm, st);
    return check_launch("k_canonical");
}
}  // namespace

void set_force_exact(int v) { g_force_exact = v; }

int last_distance_stats(int64_t *pairs, int64_t *rechecked, int64_t *exact)
{
    if (pairs) *pairs = t_pairs;
    if (rechecked) *rechecked = t_rechecked;
    if (exact) *exact = t_exact;
    return CIL_OK;
}

// Bins / counts for all pairs.  hist_host[M+1] gets the per-bin pair counts.
template <typename T>
int pair_bins_impl(const T *A, long long nA, const T *B, long long nB, long long dim,
                   const double *radii, int M, uint8_t *bins, std::vector<unsigned long long> &hist_host,
                   hipStream_t st)
{
    const long long npairs = nA * nB;
    DistScratch s;
    CIL_TRY(scratch(npairs, &s));
    std::vector<double> thr(M);
    for (int m = 0; m < M; ++m) thr[m] = radii[m] * radii[m];
    CIL_HIP(hipMemcpyAsync(s.thr, thr.data(), sizeof(double) * M, hipMemcpyHostToDevice, st));
    CIL_TRY(fill_zero(s.hist, sizeof(unsigned long long) * (M + 1), st));
    CIL_TRY(fill_zero(s.nrecheck, sizeof(unsigned long long) * 2, st));

    BinOut o{};
    o.thr = s.thr;
    o.M = M;
    o.eps_rel = (double)(dim + 4) * 0x1p-53 * 1.01;
    o.hist = s.hist;
    o.bins = bins;
    o.recheck = s.recheck;
    o.nrecheck = s.nrecheck;
    o.recheck_cap = s.cap;
    if (npairs > 0) {
        const ProfMark pm = prof_begin("k_dist_tile", st);
        hipLaunchKernelGGL((k_dist_tile<T, false>), tile_grid(nA, nB), dim3(256), 0, st, A, nA, B, nB, dim, o);
        prof_end(pm, st);
        CIL_TRY(check_launch("k_dist_tile"));
    }
    unsigned long long nre = 0;
    CIL_HIP(hipMemcpyAsync(&nre, s.nrecheck, sizeof(nre), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    if ((long long)nre > s.cap) return set_error(CIL_EDEVICE, "re-check list overflow");
    CanonOut co{};
    co.pairs = s.recheck;
    co.npairs_dev = s.nrecheck;
    co.cap = s.cap;
    co.thr = s.thr;
    co.M = M;
    co.hist = s.hist;
    co.bins = bins;
    co.nB = nB;
    co.nexact = s.nexact;
    co.force_exact = g_force_exact;
    CIL_TRY(run_canonical(A, B, dim, co, (long long)nre, st));
    hist_host.assign(M + 1, 0);
    unsigned long long nex = 0;
    CIL_HIP(hipMemcpyAsync(hist_host.data(), s.hist, sizeof(unsigned long long) * (M + 1),
                           hipMemcpyDeviceToHost, st));
    CIL_HIP(hipMemcpyAsync(&nex, s.nexact, sizeof(nex), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    t_pairs = npairs;
    t_rechecked = (long long)nre;
    t_exact = (long long)nex;
    return CIL_OK;
}

template int pair_bins_impl<double>(const double *, long long, const double *, long long, long long,
                                    const double *, int, uint8_t *, std::vector<unsigned long long> &,
                                    hipStream_t);
template int pair_bins_impl<float>(const float *, long long, const float *, long long, long long,
                                   const double *, int, uint8_t *, std::vector<unsigned long long> &,
                                   hipStream_t);

template <typename T>
int distance_range_impl(const T *A, long long nA, const T *B, long long nB, long long dim, int excl,
                        double *dmin, double *dmax, hipStream_t st)
{
    const long long npairs = nA * nB;
    DistScratch s;
    CIL_TRY(scratch(npairs, &s));
    void *p;
    CIL_TRY(ws_get(WS_DIST_SAMPLE, sizeof(double) * (size_t)std::max<long long>(npairs, 1), &p));
    double *dmat = (double *)p;
    unsigned long long init[2] = {(unsigned long long)0x7ff0000000000000ull, 0ull};   // +inf, 0
    CIL_HIP(hipMemcpyAsync(s.minmax, init, sizeof(init), hipMemcpyHostToDevice, st));
    CIL_TRY(fill_zero(s.nrecheck, sizeof(unsigned long long) * 2, st));
    BinOut o{};
    o.dmat = dmat;
    o.exclude_diag = excl;
    o.dmin_bits = s.minmax;
    o.dmax_bits = s.minmax + 1;
    const ProfMark pm = prof_begin("k_dist_tile_range", st);
    hipLaunchKernelGGL((k_dist_tile<T, true>), tile_grid(nA, nB), dim3(256), 0, st, A, nA, B, nB, dim, o);
    prof_end(pm, st);
    CIL_TRY(check_launch("k_dist_tile range"));
    unsigned long long mm[2];
    CIL_HIP(hipMemcpyAsync(mm, s.minmax, sizeof(mm), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    double fmin_, fmax_;
    memcpy(&fmin_, &mm[0], 8);
    memcpy(&fmax_, &mm[1], 8);
    if (!std::isfinite(fmin_) || !std::isfinite(fmax_))
        return set_error(CIL_ENONFINITE, "non-finite distances in range computation");
    const double eps = (double)(dim + 4) * 0x1p-53 * 1.01;
    const double lo_thr = fmin_ * (1.0 + 2.0 * eps) + 1e-300;
    const double hi_thr = fmax_ * (1.0 - 2.0 * eps);
    const long long nthr = 256;
    hipLaunchKernelGGL(k_range_candidates, dim3((unsigned)((npairs + nthr - 1) / nthr)), dim3(nthr), 0, st,
                       (const double *)dmat, nA, nB, lo_thr, hi_thr, excl, s.recheck, s.nrecheck, s.cap);
    CIL_TRY(check_launch("k_range_candidates"));
    unsigned long long nc = 0;
    CIL_HIP(hipMemcpyAsync(&nc, s.nrecheck, sizeof(nc), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    if ((long long)nc > s.cap) return set_error(CIL_EDEVICE, "range candidate overflow");
    double *cand;
    CIL_TRY(ws_get(WS_DIST_NORMS, sizeof(double) * std::max<unsigned long long>(nc, 1), (void **)&cand));
    CanonOut co{};
    co.pairs = s.recheck;
    co.npairs_dev = s.nrecheck;
    co.cap = s.cap;
    co.d2 = cand;
    co.nexact = s.nexact;
    co.force_exact = g_force_exact;
    CIL_TRY(run_canonical(A, B, dim, co, (long long)nc, st));
    std::vector<double> hc(nc);
    if (nc) CIL_HIP(hipMemcpyAsync(hc.data(), cand, sizeof(double) * nc, hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    double lo = INFINITY, hi = 0.0;
    for (double v : hc) {
        lo = std::min(lo, v);
        hi = std::max(hi, v);
    }
    *dmin = lo;
    *dmax = hi;
    t_pairs = npairs;
    t_rechecked = (long long)nc;
    return CIL_OK;
}

template int distance_range_impl<double>(const double *, long long, const double *, long long, long long,
                                         int, double *, double *, hipStream_t);
template int distance_range_impl<float>(const float *, long long, const float *, long long, long long, int,
                                        double *, double *, hipStream_t);

template <typename T>
int canonical_pairs_impl(const T *A, long long nA, const T *B, long long nB, long long dim, const long long *ia,
                         const long long *jb, long long np, double *d2, hipStream_t st)
{
    DistScratch s;
    CIL_TRY(scratch(1, &s));
    // nrecheck slot doubles as the bad-index flag here; nexact counts fallbacks
    CIL_TRY(fill_zero(s.nrecheck, sizeof(unsigned long long) * 2, st));
    CanonOut co{};
    co.ia = ia;
    co.jb = jb;
    co.npairs = np;
    co.nA = nA;
    co.nB = nB;
    co.bad = (int *)s.nrecheck;
    co.d2 = d2;
    co.nexact = s.nexact;
    co.force_exact = g_force_exact;
    CIL_TRY(run_canonical(A, B, dim, co, np, st));
    unsigned long long flags[2];
    CIL_HIP(hipMemcpyAsync(flags, s.nrecheck, sizeof(flags), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    t_pairs = np;
    t_rechecked = np;
    t_exact = (long long)flags[1];
    if (flags[0]) return set_error(CIL_EINVAL, "pair index out of range");
    return CIL_OK;
}

template int canonical_pairs_impl<double>(const double *, long long, const double *, long long, long long,
                                          const long long *, const long long *, long long, double *, hipStream_t);
template int canonical_pairs_impl<float>(const float *, long long, const float *, long long, long long,
                                         const long long *, const long long *, long long, double *, hipStream_t);

}  // namespace cil
