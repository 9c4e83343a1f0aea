// Pair distances, radius bins and correlation sums (Sec. 2.1, eqs. eCDF and
// CIL) on gfx950.
//
// Canonical squared distance of two patterns a, b of length d:
//   d_k = fl64(a_k - b_k)  (inputs converted to double),
//   D   = RN64(sum_k d_k^2)   -- the exact sum, rounded once.
// Counting rule: a pair lies under radius R_m when D < fl(R_m * R_m).
//
// Pipeline for every pair statistic:
//   1. fast pass -> FP64 partials P[split][i][j] over K ranges:
//      FP64 sets: direct differences, P = sum d_k^2 over the range (k_dist_partial);
//      FP32 sets: split-bf16x3 Gram on the matrix cores (gram.hip).
//   2. k_classify sums the partials in a fixed order into D~ and its rigorous
//      bound eps (direct: all terms are non-negative, so any summation order
//      is within gamma_{d+S} D~ of the exact sum, and eps = (d + S + 4)
//      2^-53 1.01 D~; Gram: the bound derived in gram.hip), then bins the pair
//      or, when |D~ - fl(R_m^2)| <= eps for some m, puts it on a re-check list.
//   3. k_canonical recomputes the listed pairs canonically; every count is exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cil_internal.hpp"
#include "distance_async.hpp"
#include "radii_dd.hpp"

// The error-free transformations below (two-sum, exact squares split by an
// FMA) are only exact if no product is fused into a later sum: contraction
// off for this file; the fused multiply-adds that are wanted are explicit.
#pragma clang fp contract(off)

namespace cil {

// gram.hip
struct GramWork {
    __bf16 *Ah, *Al, *Bh, *Bl;
    double *na, *nb;
    float *c;
    long long dimP;
};
int gram_prepare(const float *, long long, const float *, long long, long long, GramWork *, hipStream_t);
long long gram_splits(long long, long long, long long);
int gram_partials(const GramWork &, long long, long long, long long, long long, double *, hipStream_t);

constexpr int TILE = 64;       // pairs per tile side (direct pass)
constexpr int KC = 16;         // k-chunk staged in LDS
constexpr int MAX_M = 255;

__device__ __forceinline__ double ld(const double *p) { return *p; }
__device__ __forceinline__ double ld(const float *p) { return (double)*p; }

// ------------------------------------------------------------ direct pass
// One 64 x 64 tile of pairs and one K range per block of 256 threads; thread
// (ty, tx) owns rows ty + 16 i and columns tx + 16 j, i, j < 4.
template <typename T>
__global__ __launch_bounds__(256) void k_dist_partial(const T *A, long long nA, const T *B, long long nB,
                                                      long long dim, long long ksplit, double *P)
{
    __shared__ double sA[TILE][KC + 1];
    __shared__ double sB[TILE][KC + 1];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const long long i0 = (long long)blockIdx.y * TILE, j0 = (long long)blockIdx.x * TILE;
    const long long kb = (long long)blockIdx.z * ksplit;
    const long long ke = kb + ksplit < dim ? kb + ksplit : dim;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (long long k0 = kb; k0 < ke; k0 += KC) {
        __syncthreads();
        for (int e = tid; e < TILE * KC; e += 256) {
            const int r = e / KC, kk = e % KC;
            const long long k = k0 + kk;
            const long long ia = i0 + r, jb = j0 + r;
            sA[r][kk] = (ia < nA && k < ke) ? ld(A + ia * dim + k) : 0.0;
            sB[r][kk] = (jb < nB && k < ke) ? ld(B + jb * dim + k) : 0.0;
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
    double *Ps = P + (long long)blockIdx.z * nA * nB;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long ia = i0 + ty + 16 * i, jb = j0 + tx + 16 * j;
            if (ia < nA && jb < nB) Ps[ia * nB + jb] = acc[i][j];
        }
}

// ---------------------------------------------------------------- classify
enum { MODE_BINS = 0, MODE_RANGE1 = 1, MODE_RANGE2 = 2, MODE_DUMP = 3 };

struct ClassifyArgs {
    const double *P;            // partials [S][nA][nB]
    int S;
    int gram;                   // 0: direct partials of D, 1: Gram partials
    const double *na, *nb;      // Gram: |a^|^2, |b^|^2
    double eps_rel;             // direct
    double eG;                  // Gram: eG / (|a'||b'|)
    double e1;                  // Gram: split error per element
    int mode;
    int exclude_diag;
    const double *thr;          // bins: [M]
    double thr_slack;           // bins: also list the pairs within thr_slack thr of a threshold
    int M;
    unsigned long long *hist;   // bins: [M+1]
    uint8_t *bins;              // bins: [nA][nB] or null
    int2 *list;                 // re-check / candidate list
    unsigned long long *nlist;
    long long cap;
    unsigned long long *minmax; // range: [min(D~+eps) bits, max(D~-eps) bits]
    unsigned long long *flag;   // range: set when a distance is not finite
    double *reduced;            // range pass 1: the summed partials of every pair, or null
    double *dump_d, *dump_eps;  // dump
};

__device__ __forceinline__ void approx_pair(const ClassifyArgs &c, long long i, long long j, long long nA,
                                            long long nB, double &D, double &eps)
{
    double s = 0.0;
    const double *pp = c.P + i * nB + j;
    const long long ps = nA * nB;
    int k = 0;
    for (; k + 8 <= c.S; k += 8) {               // eight loads in flight, added in order
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pp[(k + u) * ps];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; k < c.S; ++k) s += pp[k * ps];
    // the sum of the partials, for the later passes (0 + s is s exactly, so
    // they see the same D~ from one partial)
    if (c.reduced) c.reduced[i * nB + j] = s;
    if (!c.gram) {
        D = s;
        eps = c.eps_rel * s;
        return;
    }
    const double na = c.na[i], nb = c.nb[j];
    D = na + nb - 2.0 * s;
    const double ra = sqrt(na), rb = sqrt(nb);
    const double Sg = ra + rb;
    const double eG = c.eG * ra * rb;
    const double Dp = D > 0.0 ? D : 0.0;
    const double u = 0x1p-53;
    const double bound = 2.0 * eG + 2.0 * c.e1 * Sg * (sqrt(Dp + 2.0 * eG) + c.e1 * Sg) + c.e1 * c.e1 * Sg * Sg +
                         8.0 * u * (na + nb + Dp) + u * Dp;
    eps = 2.0 * bound;
}

__global__ __launch_bounds__(256) void k_classify(ClassifyArgs c, long long nA, long long nB)
{
    __shared__ unsigned int hist[MAX_M + 1];
    __shared__ double sthr[MAX_M];
    __shared__ unsigned long long rlo[4], rhi[4];
    __shared__ int rbad[4];
    const int tid = threadIdx.x;
    if (c.mode == MODE_BINS) {
        for (int m = tid; m <= c.M; m += 256) hist[m] = 0;
        for (int m = tid; m < c.M; m += 256) sthr[m] = c.thr[m];
        __syncthreads();
    }
    const long long n = nA * nB;
    unsigned long long lo = ~0ull, hi = 0ull;     // RANGE1: bounds over this thread's pairs
    int bad = 0;
    // grid-stride over the pairs (the grid is capped, so per-block reductions stay few)
    for (long long e = (long long)blockIdx.x * 256 + tid; e < n; e += (long long)gridDim.x * 256) {
        const long long i = e / nB, j = e % nB;
        if (c.exclude_diag && i == j && !c.reduced) continue;
        double D, eps;
        approx_pair(c, i, j, nA, nB, D, eps);
        if (c.exclude_diag && i == j) continue;     // summed for the later passes, not part of the range
        const bool finite = isfinite(D) && isfinite(eps);
        if (c.mode == MODE_BINS) {
            int bin = 0;
            bool amb = !finite;
            for (int m = 0; m < c.M; ++m) {
                const double t = sthr[m];
                if (fabs(D - t) <= eps + c.thr_slack * t) amb = true;
                bin += (D < t);
            }
            if (amb) {
                const unsigned long long slot = atomicAdd(c.nlist, 1ull);
                if ((long long)slot < c.cap) c.list[slot] = make_int2((int)i, (int)j);
            } else {
                atomicAdd(&hist[bin], 1u);
                if (c.bins) c.bins[i * nB + j] = (uint8_t)bin;
            }
        } else if (c.mode == MODE_RANGE1) {
            // the bit patterns of non-negative doubles order as the values
            if (!finite) {
                bad = 1;
            } else {
                const unsigned long long l = (unsigned long long)__double_as_longlong(D + eps);
                const unsigned long long h = (unsigned long long)__double_as_longlong(fmax(D - eps, 0.0));
                lo = l < lo ? l : lo;
                hi = h > hi ? h : hi;
            }
        } else if (c.mode == MODE_RANGE2) {
            const double mnub = __longlong_as_double((long long)c.minmax[0]);
            const double mxlb = __longlong_as_double((long long)c.minmax[1]);
            if (D - eps <= mnub || D + eps >= mxlb) {
                const unsigned long long slot = atomicAdd(c.nlist, 1ull);
                if ((long long)slot < c.cap) c.list[slot] = make_int2((int)i, (int)j);
            }
        } else {
            c.dump_d[e] = D;
            c.dump_eps[e] = eps;
        }
    }
    if (c.mode == MODE_BINS) {
        __syncthreads();
        for (int m = tid; m <= c.M; m += 256)
            if (hist[m]) atomicAdd(&c.hist[m], (unsigned long long)hist[m]);
    } else if (c.mode == MODE_RANGE1) {
        // wavefront, then workgroup, then one atomic per workgroup
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long l2 = __shfl_xor(lo, o, 64), h2 = __shfl_xor(hi, o, 64);
            lo = l2 < lo ? l2 : lo;
            hi = h2 > hi ? h2 : hi;
            bad |= __shfl_xor(bad, o, 64);
        }
        if ((tid & 63) == 0) {
            rlo[tid >> 6] = lo;
            rhi[tid >> 6] = hi;
            rbad[tid >> 6] = bad;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < 4; ++w) {
                lo = rlo[w] < lo ? rlo[w] : lo;
                hi = rhi[w] > hi ? rhi[w] : hi;
                bad |= rbad[w];
            }
            if (bad) atomicOr(c.flag, 1ull);          // a non-finite distance
            if (lo != ~0ull) atomicMin(&c.minmax[0], lo);
            if (hi != 0ull) atomicMax(&c.minmax[1], hi);
        }
    }
}

// ---------------------------------------------------------------- canonical
// Double-double accumulation of the exact squares, one wavefront per pair (or
// sixteen, when few pairs are re-checked), then a certified rounding.  The accumulation records whether any of its
// roundings lost bits: if none did, hi + lo is the exact sum and the
// hardware's RN(hi + lo) is the correctly rounded value, ties included (the
// common case for FP32 sets, whose squares are exact).  Otherwise, with the
// relative error bound delta, RN(sum) = RN(hi + lo) whenever the interval
// [S - delta S, S + delta S] holds no rounding boundary.  If neither holds
// (or when forced) the wavefront recomputes the sum exactly: each lane builds
// a non-overlapping expansion of its terms (Shewchuk's exact summation),
// lane 0 merges the 64 expansions and rounds once, half to even.

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += (bh, bl); inexact |= some rounding lost bits
__device__ __forceinline__ void dd_add_t(double &hi, double &lo, double bh, double bl, int &inexact)
{
    double s, e, t, et, u, eu;
    two_sum(hi, bh, s, e);
    two_sum(lo, bl, t, et);
    two_sum(e, t, u, eu);
    inexact |= (et != 0.0) | (eu != 0.0);
    hi = s + u;
    lo = u - (hi - s);
}

constexpr int EXP_CAP = 64;     // a non-overlapping expansion of doubles has < 40 parts

__device__ __forceinline__ void exp_add(double (&part)[EXP_CAP], int &np, double x)
{
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
}

__device__ __forceinline__ double exp_round(const double (&part)[EXP_CAP], int np)
{
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

// Exact sum over the wavefront (all 64 lanes call it); result valid in lane 0.
template <typename T>
__device__ double exact_d2_wave(const T *a, const T *b, long long dim, int lane)
{
    double part[EXP_CAP];
    int np = 0;
    for (long long k = lane; k < dim; k += 64) {
        const double d = ld(a + k) - ld(b + k);
        const double p = d * d;
        const double e = fma(d, d, -p);
        exp_add(part, np, p);
        if (e != 0.0) exp_add(part, np, e);
    }
    int maxm = np;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) maxm = max(maxm, __shfl_xor(maxm, o, 64));
    for (int src = 1; src < 64; ++src) {
        for (int c = 0; c < maxm; ++c) {
            const double mine = c < np ? part[c] : 0.0;
            const double v = __shfl(mine, src, 64);
            if (lane == 0 && v != 0.0) exp_add(part, np, v);
        }
    }
    return lane == 0 ? exp_round(part, np) : 0.0;
}

struct CanonOut {
    // pair source: either an int2 list (recheck) or two index arrays
    const int2 *pairs;
    const unsigned long long *npairs_dev;   // count for the list (clamped to cap)
    long long cap;
    long long first;            // list mode: the launch covers pairs first, first + 1, ...
    long long stride;           // list mode: > 0 loops each wave (WPP 1) or block over w, w + stride, ...
    const long long *ia, *jb;
    long long npairs;
    long long nA;               // index bounds for the ia/jb source
    int *bad;                   // set when an ia/jb index is out of range
    // sinks
    double *d2;                 // per pair, or null
    unsigned long long *range_mm;   // or null: [0] min, [1] max of the pairs' D (bits of non-negative doubles)
    const double *thr;
    int M;
    unsigned long long *hist;   // or null
    uint8_t *bins;              // or null
    double win_rel;             // with win_hits: bit m set when a pair lies within win_rel thr[m] of thr[m]
    unsigned long long *win_hits;
    long long nB;
    unsigned long long *nexact;
    int force_exact;
};

// WPP wavefronts per pair: 1 (four pairs per 256-thread block; many pairs, the
// pass is bandwidth-bound) or 16 (one pair per 1024-thread block; few pairs,
// latency-bound).  The certified rounding makes the result independent of
// the summation order, so both give the same doubles.
template <typename T, int WPP>
__device__ __forceinline__ void canonical_pair(const T *A, const T *B, long long dim, const CanonOut &o, long long w,
                                               int lane, int sub);

template <typename T, int WPP>
__global__ __launch_bounds__(WPP == 1 ? 256 : 64 * WPP) void k_canonical(const T *A, const T *B, long long dim,
                                                                         CanonOut o)
{
    const int lane = threadIdx.x & 63;
    const int sub = WPP == 1 ? 0 : threadIdx.x / 64;
    // list mode: the grid may be sized before the list count is known (an
    // upper bound); waves past the count leave at once, or with a stride
    // (the grid's pair slots) each wave or block takes every stride-th pair
    const long long w = (WPP == 1 ? (long long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64
                                  : (long long)blockIdx.x) + (o.pairs ? o.first : 0);
    const long long np = o.pairs ? (long long)min((unsigned long long)o.cap, *o.npairs_dev) : o.npairs;
    if (o.pairs && o.stride > 0) {       // the trip count is uniform over a block
        for (long long v = w; v < np; v += o.stride) {
            canonical_pair<T, WPP>(A, B, dim, o, v, lane, sub);
            if constexpr (WPP > 1) __syncthreads();   // wave 0 is done with the pair's partials
        }
        return;
    }
    if (w >= np) return;
    canonical_pair<T, WPP>(A, B, dim, o, w, lane, sub);
}

// The canonical squared distance of pair w (of the list or the index arrays)
// and its sinks, by one wave (WPP 1) or the block's WPP waves.
template <typename T, int WPP>
__device__ __forceinline__ void canonical_pair(const T *A, const T *B, long long dim, const CanonOut &o, long long w,
                                               int lane, int sub)
{
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
    int inexact = 0;
    // four strides' loads in flight; terms accumulated in the same order
    constexpr long long STR = 64LL * WPP;
    long long k = lane + 64LL * sub;
    for (; k + 3 * STR < dim; k += 4 * STR) {
        double da[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) da[u] = ld(a + k + u * STR) - ld(b + k + u * STR);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double p = da[u] * da[u];
            dd_add_t(hi, lo, p, fma(da[u], da[u], -p), inexact);
        }
    }
    for (; k < dim; k += STR) {
        const double d = ld(a + k) - ld(b + k);
        const double p = d * d;
        dd_add_t(hi, lo, p, fma(d, d, -p), inexact);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double oh = __shfl_xor(hi, off, 64), ol = __shfl_xor(lo, off, 64);
        dd_add_t(hi, lo, oh, ol, inexact);
        inexact |= __shfl_xor(inexact, off, 64);
    }
    if constexpr (WPP > 1) {      // combine the pair's wavefronts; wavefront 0 finishes
        __shared__ double phi[WPP], plo[WPP];
        __shared__ int pin[WPP];
        if (lane == 0) {
            phi[sub] = hi;
            plo[sub] = lo;
            pin[sub] = inexact;
        }
        __syncthreads();
        if (sub != 0) return;
        for (int v = 1; v < WPP; ++v) {
            dd_add_t(hi, lo, phi[v], plo[v], inexact);
            inexact |= pin[v];
        }
    }
    double R, e;
    two_sum(hi, lo, R, e);
    const double delta = (double)(dim + 65 * WPP + 64) * 0x1p-100;   // relative error bound
    int ex;
    const double frac = frexp(R, &ex);                   // R = frac 2^ex, frac in [0.5, 1)
    // rounding boundaries of R: R +- half an ulp (ulp = 2^(ex-53)), except
    // below a power of two, where the spacing halves
    const double half = (e < 0.0 && frac == 0.5) ? ldexp(1.0, ex - 55) : ldexp(1.0, ex - 54);
    int certain = isfinite(R) && (!inexact || fabs(e) + delta * R < half || R == 0.0);
    certain = __shfl(certain, 0, 64);                    // lane 0 decides for the wavefront
    double D = R;
    if (!certain || o.force_exact) {
        D = exact_d2_wave(a, b, dim, lane);
        if (lane == 0) atomicAdd(o.nexact, 1ull);
    }
    if (lane == 0) {
        if (o.d2) o.d2[w] = D;
        if (o.range_mm) {       // non-negative doubles order as their bit patterns
            atomicMin(&o.range_mm[0], (unsigned long long)__double_as_longlong(D));
            atomicMax(&o.range_mm[1], (unsigned long long)__double_as_longlong(D));
        }
        if (o.hist) {
            int bin = 0;
            unsigned long long near = 0;
            for (int m = 0; m < o.M; ++m) {
                bin += (D < o.thr[m]);
                if (o.win_hits && fabs(D - o.thr[m]) <= o.win_rel * o.thr[m]) near |= 1ull << m;
            }
            atomicAdd(&o.hist[bin], 1ull);
            if (near) atomicOr(o.win_hits, near);
            if (o.bins) o.bins[i * o.nB + j] = (uint8_t)bin;
        }
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
    unsigned long long *nlist = nullptr;
    unsigned long long *nexact = nullptr;
    unsigned long long *minmax = nullptr;
    unsigned long long *flag = nullptr;
    unsigned long long *cmm = nullptr;      // canonical extremes of the range candidates (bits)
    RangeOut *ro = nullptr;
    int2 *list = nullptr;
    long long cap = 0;
};

int scratch(long long cap, DistScratch *s)
{
    void *p;
    CIL_TRY(ws_get(WS_DIST_MISC, 4096 + sizeof(double) * 512, &p));
    char *c = (char *)p;
    s->thr = (double *)c;                                   // 256 doubles
    s->hist = (unsigned long long *)(c + 2048);             // 256 counters
    s->nlist = (unsigned long long *)(c + 4096);
    s->nexact = s->nlist + 1;
    s->minmax = s->nlist + 2;
    s->flag = s->nlist + 4;
    s->cmm = s->nlist + 5;
    s->ro = (RangeOut *)(c + 4096 + 64);
    static_assert(4096 + 64 + sizeof(RangeOut) <= 4096 + sizeof(double) * 512, "range output fits the workspace");
    CIL_TRY(ws_get(WS_DIST_RECHECK, sizeof(int2) * (size_t)std::max<long long>(cap, 1), &p));
    s->list = (int2 *)p;
    s->cap = cap;
    return CIL_OK;
}

// Launches waves for pairs co.first .. co.first + nwaves - 1 (in list mode
// nwaves may exceed the list: the surplus waves leave at once).
template <typename T>
int run_canonical(const T *A, const T *B, long long dim, CanonOut &co, long long nwaves, hipStream_t st)
{
    if (nwaves <= 0) return CIL_OK;
    const ProfMark pm = prof_begin("k_canonical", st);
    if (nwaves < 2048 && dim >= 4096)
        hipLaunchKernelGGL((k_canonical<T, 16>), dim3((unsigned)nwaves), dim3(1024), 0, st, A, B, dim, co);
    else
        hipLaunchKernelGGL((k_canonical<T, 1>), dim3((unsigned)((nwaves + 3) / 4)), dim3(256), 0, st, A, B, dim, co);
    prof_end(pm, st);
    return check_launch("k_canonical");
}

struct Approx {
    ClassifyArgs c{};
};

// Re-check launches are sized before the host knows the list's length: an
// upper bound covers the usual case in the same stream pass, and only a
// longer list costs a second launch after the count is read back.
long long recheck_guess(long long dim) { return dim >= 4096 ? 256 : 2048; }

// FP64 sets: direct differences, split over K so the grid fills the chip.
int approx_pass(const double *A, long long nA, const double *B, long long nB, long long dim, Approx *ap,
                hipStream_t st)
{
    const long long tiles = ((nA + TILE - 1) / TILE) * ((nB + TILE - 1) / TILE);
    long long S = 1;
    while (tiles * S < 1024 && dim / (2 * S) >= 256) S *= 2;
    const long long ks = std::max<long long>(KC, (dim / S + KC - 1) / KC * KC);
    S = std::max<long long>(1, (dim + ks - 1) / ks);
    void *p;
    CIL_TRY(ws_get(WS_DIST_SAMPLE, sizeof(double) * (size_t)std::max<long long>(S * nA * nB, 1), &p));
    ap->c.P = (const double *)p;
    ap->c.S = (int)S;
    ap->c.gram = 0;
    ap->c.eps_rel = (double)(dim + S + 4) * 0x1p-53 * 1.01;
    if (nA * nB > 0) {
        dim3 grid((unsigned)((nB + TILE - 1) / TILE), (unsigned)((nA + TILE - 1) / TILE), (unsigned)S);
        const ProfMark pm = prof_begin("k_dist_partial", st);
        hipLaunchKernelGGL(k_dist_partial<double>, grid, dim3(256), 0, st, A, nA, B, nB, dim, ks, (double *)p);
        prof_end(pm, st);
        CIL_TRY(check_launch("k_dist_partial"));
    }
    return CIL_OK;
}

// FP32 sets: split-bf16x3 Gram on the matrix cores.
int approx_pass(const float *A, long long nA, const float *B, long long nB, long long dim, Approx *ap,
                hipStream_t st)
{
    GramWork g;
    CIL_TRY(gram_prepare(A, nA, B, nB, dim, &g, st));
    long long S = gram_splits(nA, nB, g.dimP);
    const long long ks = std::max<long long>(64, (g.dimP / S + 63) / 64 * 64);
    S = std::max<long long>(1, (g.dimP + ks - 1) / ks);
    void *p;
    CIL_TRY(ws_get(WS_DIST_SAMPLE, sizeof(double) * (size_t)std::max<long long>(S * nA * nB, 1), &p));
    ap->c.P = (const double *)p;
    ap->c.S = (int)S;
    ap->c.gram = 1;
    ap->c.na = g.na;
    ap->c.nb = g.nb;
    ap->c.eG = 3.0 * (double)gram_flush_interval() * 0x1p-24 + 0x1p-18 + 0x1p-40;
    ap->c.e1 = 0x1p-24 + 0x1p-18;
    if (nA * nB > 0) CIL_TRY(gram_partials(g, nA, nB, S, ks, (double *)p, st));
    return CIL_OK;
}

int classify(ClassifyArgs &c, long long nA, long long nB, hipStream_t st)
{
    const long long n = nA * nB;
    if (n <= 0) return CIL_OK;
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    static const char *const names[] = {"k_classify_bins", "k_classify_range1", "k_classify_range2", "k_classify_dump"};
    const ProfMark pm = prof_begin(names[c.mode], st);
    hipLaunchKernelGGL(k_classify, dim3((unsigned)blocks), dim3(256), 0, st, c, nA, nB);
    prof_end(pm, st);
    return check_launch("k_classify");
}
}  // namespace

void set_force_exact(int v) { g_force_exact = v; }

void set_distance_stats(long long pairs, long long rechecked, long long exact)
{
    t_pairs = pairs;
    t_rechecked = rechecked;
    t_exact = exact;
}

int last_distance_stats(int64_t *pairs, int64_t *rechecked, int64_t *exact)
{
    if (pairs) *pairs = t_pairs;
    if (rechecked) *rechecked = t_rechecked;
    if (exact) *exact = t_exact;
    return CIL_OK;
}

// Bins / counts for all pairs.  hist_host[M+1] gets the per-bin pair counts.
namespace {

// Bins of every pair from a computed fast pass: classify against the squared
// radii, re-check the listed pairs canonically.  hist_host[m] = #{bin == m}.
template <typename T>
int bins_from_approx(const T *A, long long nA, const T *B, long long nB, long long dim, Approx &ap, DistScratch &s,
                     const double *radii, int M, uint8_t *bins, std::vector<unsigned long long> &hist_host,
                     hipStream_t st)
{
    // pinned staging: [0, 2048) thresholds, [2048, 4096) histogram, [4096, 4112) counters
    char *hs;
    CIL_TRY(host_stage(HS_DIST, 4096 + 64, (void **)&hs));
    double *thr = (double *)hs;
    for (int m = 0; m < M; ++m) thr[m] = radii[m] * radii[m];
    CIL_HIP(hipMemcpyAsync(s.thr, thr, sizeof(double) * M, hipMemcpyHostToDevice, st));
    // the histogram and the two list counters (contiguous) in one clear
    CIL_TRY(fill_zero(s.hist, (char *)(s.nlist + 2) - (char *)s.hist, st));
    ClassifyArgs &c = ap.c;
    c.mode = MODE_BINS;
    c.thr = s.thr;
    c.M = M;
    c.hist = s.hist;
    c.bins = bins;
    c.list = s.list;
    c.nlist = s.nlist;
    c.cap = s.cap;
    CIL_TRY(classify(c, nA, nB, st));
    CanonOut co{};
    co.pairs = s.list;
    co.npairs_dev = s.nlist;
    co.cap = s.cap;
    co.thr = s.thr;
    co.M = M;
    co.hist = s.hist;
    co.bins = bins;
    co.nB = nB;
    co.nexact = s.nexact;
    co.force_exact = g_force_exact;
    const long long guess = std::min(recheck_guess(dim), std::max(s.cap, 1LL));
    CIL_TRY(run_canonical(A, B, dim, co, guess, st));
    unsigned long long *hh = (unsigned long long *)(hs + 2048);
    unsigned long long *cnt = (unsigned long long *)(hs + 4096);   // listed pairs, exact fallbacks
    CIL_HIP(hipMemcpyAsync(hh, s.hist, sizeof(unsigned long long) * (M + 1), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipMemcpyAsync(cnt, s.nlist, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    CIL_TRY(stream_wait(st));
    const unsigned long long nre = cnt[0];
    if ((long long)nre > s.cap) return set_error(CIL_EDEVICE, "re-check list overflow");
    if ((long long)nre > guess) {                       // the rest of a long list
        co.first = guess;
        CIL_TRY(run_canonical(A, B, dim, co, (long long)nre - guess, st));
        CIL_HIP(hipMemcpyAsync(hh, s.hist, sizeof(unsigned long long) * (M + 1), hipMemcpyDeviceToHost, st));
        CIL_HIP(hipMemcpyAsync(cnt, s.nlist, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        CIL_TRY(stream_wait(st));
    }
    hist_host.assign(hh, hh + M + 1);
    t_pairs = nA * nB;
    t_rechecked = (long long)nre;
    t_exact = (long long)cnt[1];
    return CIL_OK;
}

// Canonical extremes from a computed fast pass: pass 1 bounds them by
// min(D~ + eps) and max(D~ - eps); pass 2 lists every pair whose interval
// reaches those bounds; the listed pairs are recomputed canonically and the
// extremes taken over them.
template <typename T>
int range_from_approx(const T *A, long long nA, const T *B, long long nB, long long dim, Approx &ap, DistScratch &s,
                      int excl, double *dmin, double *dmax, hipStream_t st)
{
    const long long guess = std::min(recheck_guess(dim), std::max(s.cap, 1LL));
    // pinned staging: [0, 40) initial counters, [64, 104) counters read back,
    // [4096, ...) candidate distances read back
    char *hs;
    CIL_TRY(host_stage(HS_DIST, 4096 + sizeof(double) * (size_t)guess, (void **)&hs));
    unsigned long long *init = (unsigned long long *)hs;
    // nlist, nexact, min bound (+inf), max bound (0), non-finite flag
    init[0] = 0ull;
    init[1] = 0ull;
    init[2] = (unsigned long long)0x7ff0000000000000ull;
    init[3] = 0ull;
    init[4] = 0ull;
    CIL_HIP(hipMemcpyAsync(s.nlist, init, 5 * sizeof(unsigned long long), hipMemcpyHostToDevice, st));
    ClassifyArgs &c = ap.c;
    c.exclude_diag = excl;
    c.minmax = s.minmax;
    c.flag = s.flag;
    c.list = s.list;
    c.nlist = s.nlist;
    c.cap = s.cap;
    // pass 1 reads every partial once and leaves their sums, so that pass 2
    // and the bins read one value per pair
    if (c.S > 1) CIL_TRY(ws_get(WS_DIST_REDUCED, sizeof(double) * (size_t)std::max(nA * nB, 1LL), (void **)&c.reduced));
    c.mode = MODE_RANGE1;
    CIL_TRY(classify(c, nA, nB, st));
    if (c.reduced) {
        c.P = c.reduced;
        c.S = 1;
        c.reduced = nullptr;
    }
    c.mode = MODE_RANGE2;                 // stream-ordered after the bounds of pass 1
    CIL_TRY(classify(c, nA, nB, st));
    double *cand;
    CIL_TRY(ws_get(WS_DIST_NORMS, sizeof(double) * (size_t)guess, (void **)&cand));
    CanonOut co{};
    co.pairs = s.list;
    co.npairs_dev = s.nlist;
    co.cap = s.cap;
    co.d2 = cand;
    co.nexact = s.nexact;
    co.force_exact = g_force_exact;
    CIL_TRY(run_canonical(A, B, dim, co, guess, st));
    double *hcp = (double *)(hs + 4096);
    unsigned long long *cnt = (unsigned long long *)(hs + 64);
    CIL_HIP(hipMemcpyAsync(hcp, cand, sizeof(double) * guess, hipMemcpyDeviceToHost, st));
    CIL_HIP(hipMemcpyAsync(cnt, s.nlist, 5 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    CIL_TRY(stream_wait(st));
    std::vector<double> hc(hcp, hcp + guess);
    if (cnt[4]) return set_error(CIL_ENONFINITE, "non-finite distances in range computation");
    const long long nc = (long long)cnt[0];
    if (nc > s.cap) return set_error(CIL_EDEVICE, "range candidate overflow");
    if (nc > guess) {                     // the rest of a long candidate list
        CIL_TRY(ws_get(WS_DIST_NORMS, sizeof(double) * (size_t)nc, (void **)&cand));
        co.d2 = cand;
        co.first = guess;
        CIL_TRY(run_canonical(A, B, dim, co, nc - guess, st));
        hc.resize(nc);
        CIL_HIP(hipMemcpyAsync(hc.data() + guess, cand + guess, sizeof(double) * (nc - guess), hipMemcpyDeviceToHost,
                               st));
        CIL_HIP(hipMemcpyAsync(cnt, s.nlist, 5 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        CIL_TRY(stream_wait(st));
    }
    double lo = INFINITY, hi = 0.0;
    for (long long k = 0; k < nc; ++k) {
        lo = std::min(lo, hc[k]);
        hi = std::max(hi, hc[k]);
    }
    *dmin = lo;
    *dmax = hi;
    t_pairs = nA * nB;
    t_rechecked = nc;
    t_exact = (long long)cnt[1];
    return CIL_OK;
}

}  // namespace

template <typename T>
int pair_bins_impl(const T *A, long long nA, const T *B, long long nB, long long dim, const double *radii, int M,
                   uint8_t *bins, std::vector<unsigned long long> &hist_host, hipStream_t st)
{
    DistScratch s;
    CIL_TRY(scratch(nA * nB, &s));
    Approx ap;
    CIL_TRY(approx_pass(A, nA, B, nB, dim, &ap, st));
    return bins_from_approx(A, nA, B, nB, dim, ap, s, radii, M, bins, hist_host, st);
}

// Range, radii and bins from one fast pass (the partials stay in their
// workspace between the two classifications).
template <typename T>
int adaptive_bins_impl(const T *A, long long nA, const T *B, long long nB, long long dim, int excl, int M, int law,
                       double *dmin, double *dmax, double *radii, uint8_t *bins,
                       std::vector<unsigned long long> &hist_host, hipStream_t st)
{
    DistScratch s;
    CIL_TRY(scratch(nA * nB, &s));
    Approx ap;
    CIL_TRY(approx_pass(A, nA, B, nB, dim, &ap, st));
    CIL_TRY(range_from_approx(A, nA, B, nB, dim, ap, s, excl, dmin, dmax, st));
    ap.c.exclude_diag = 0;                 // bins of every pair
    const long long nrange = t_rechecked, nrange_exact = t_exact;
    CIL_TRY(radii_ladder(*dmin, *dmax, M, law, radii));
    CIL_TRY(bins_from_approx(A, nA, B, nB, dim, ap, s, radii, M, bins, hist_host, st));
    t_rechecked += nrange;
    t_exact += nrange_exact;
    return CIL_OK;
}

// R_0 - m h rounded as two operations, as the host forms it (no contraction).
__device__ __forceinline__ double linear_radius(double R0, int m, double h)
{
#pragma clang fp contract(off)
    return R0 - (double)m * h;
}

// The device range pass's initial counters, staged in pinned host memory
// (HS_DIST, offset 0; the caller's read-back uses the same buffer further
// on): list count, exact fallbacks, classify bounds (+inf, 0), non-finite
// flag, canonical extremes (+inf, 0), thresholds with a pair near them.
int range_init_stage(unsigned long long **out)
{
    char *hs;
    CIL_TRY(host_stage(HS_DIST, 8192, (void **)&hs));
    unsigned long long *init = (unsigned long long *)hs;
    init[0] = 0ull;
    init[1] = 0ull;
    init[2] = (unsigned long long)0x7ff0000000000000ull;
    init[3] = 0ull;
    init[4] = 0ull;
    init[5] = (unsigned long long)0x7ff0000000000000ull;
    init[6] = 0ull;
    init[7] = 0ull;
    *out = init;
    return CIL_OK;
}

// Range and radii on the device from the range pass's counters (cnt: [0]
// candidates, [1] exact fallbacks, [4] non-finite flag, [5], [6] the
// candidates' canonical extremes): the ladder as the host forms it
// (cil_radii), powers by pow_dd; thr[m] = R_m^2.  A bad range leaves every
// threshold 0 and its status in ro.
__global__ void k_range_radii(const unsigned long long *cnt, long long cap, int M, int law, double *thr, RangeOut *ro)
{
    __shared__ double sR0, sb;
    __shared__ DD slogb;
    __shared__ int sst;
    __shared__ DDTables tab;
    {                                    // the series' coefficients, one per thread
        const int k = threadIdx.x;
        if (k < kLogTerms) tab.inv_odd[k] = dd_inv(2 * k + 1);
        else if (k < kLogTerms + kExpTerms) tab.inv_n[k - kLogTerms + 1] = dd_inv(k - kLogTerms + 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double lo = __longlong_as_double((long long)cnt[5]), hi = __longlong_as_double((long long)cnt[6]);
        ro->d2min = lo;
        ro->d2max = hi;
        ro->nrange = (long long)cnt[0];
        ro->nrange_exact = (long long)cnt[1];
        int st = 0;
        if (cnt[4]) st = 2;
        else if ((long long)cnt[0] > cap) st = 3;
        const double R0 = sqrt_dd(hi), RM = sqrt_dd(lo);
        if (st == 0 && !(RM > 0.0 && R0 > RM && isfinite(R0))) st = 1;
        ro->status = st;
        sst = st;
        sR0 = R0;
        DD lb{0.0, 0.0};
        sb = st != 0 ? 0.0 : (law == 0 ? root_dd(R0 / RM, M, tab, &lb) : (R0 - RM) / M);
        slogb = lb;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        double r = 0.0;
        if (sst == 0)
            r = law == 0 ? sR0 * pow_dd_from_log(slogb, (double)-(m + 1), tab) : linear_radius(sR0, m + 1, sb);
        ro->radii[m] = r;
        thr[m] = r * r;
    }
}

// Re-check launches over a list whose length stays on the device: for
// d < 4096 one launch of 2048 waves striding over it; for longer vectors a
// first launch of 256 pairs at sixteen waves each (the usual short list at
// the latency of one pair), then a strided launch of 8192 single-wave slots
// for the rest, which leaves at once when there is none.
template <typename T>
int canonical_any_length(const T *A, const T *B, long long dim, CanonOut co, long long cap, hipStream_t st)
{
    if (dim < 4096) {
        co.stride = 2048;
        return run_canonical(A, B, dim, co, 2048, st);
    }
    const long long first = std::min(recheck_guess(dim), std::max(cap, 1LL));
    CIL_TRY(run_canonical(A, B, dim, co, first, st));
    if (cap > first) {
        constexpr long long TAIL = 8192;
        co.first = first;
        co.stride = TAIL;
        const ProfMark pm = prof_begin("k_canonical", st);
        hipLaunchKernelGGL((k_canonical<T, 1>), dim3((unsigned)(TAIL / 4)), dim3(256), 0, st, A, B, dim, co);
        prof_end(pm, st);
        CIL_TRY(check_launch("k_canonical"));
    }
    return CIL_OK;
}

// The range pass without its read-back: candidates listed as in
// range_from_approx, their canonical distances folded into the device's
// extremes, then the radii and thresholds formed on the device.
template <typename T>
int range_radii_device(const T *A, long long nA, const T *B, long long nB, long long dim, Approx &ap,
                       DistScratch &s, int M, int law, hipStream_t st)
{
    unsigned long long *init;
    CIL_TRY(range_init_stage(&init));
    CIL_HIP(hipMemcpyAsync(s.nlist, init, 8 * sizeof(unsigned long long), hipMemcpyHostToDevice, st));
    ClassifyArgs &c = ap.c;
    c.exclude_diag = 0;
    c.minmax = s.minmax;
    c.flag = s.flag;
    c.list = s.list;
    c.nlist = s.nlist;
    c.cap = s.cap;
    if (c.S > 1) CIL_TRY(ws_get(WS_DIST_REDUCED, sizeof(double) * (size_t)std::max(nA * nB, 1LL), (void **)&c.reduced));
    c.mode = MODE_RANGE1;
    CIL_TRY(classify(c, nA, nB, st));
    if (c.reduced) {
        c.P = c.reduced;
        c.S = 1;
        c.reduced = nullptr;
    }
    c.mode = MODE_RANGE2;
    CIL_TRY(classify(c, nA, nB, st));
    CanonOut co{};
    co.pairs = s.list;
    co.npairs_dev = s.nlist;
    co.cap = s.cap;
    co.range_mm = s.cmm;
    co.nexact = s.nexact;
    co.force_exact = g_force_exact;
    CIL_TRY(canonical_any_length(A, B, dim, co, s.cap, st));
    hipLaunchKernelGGL(k_range_radii, dim3(1), dim3(64), 0, st, s.nlist, s.cap, M, law, s.thr, s.ro);
    return check_launch("k_range_radii");
}

// The same without the bins' read-back: the re-check list is finished on the
// device whatever its length (strided launches), and the
// histogram and list counters stay on the device for the caller's one
// read-back at the end of a longer chain (AsyncBins).  The range and its
// read-back, which the radii need, are as in adaptive_bins_impl.
template <typename T>
int adaptive_bins_async(const T *A, long long nA, const T *B, long long nB, long long dim, int M, int law,
                        int device_radii, double *dmin, double *dmax, double *radii, uint8_t *bins, AsyncBins *ab,
                        hipStream_t st)
{
    DistScratch s;
    CIL_TRY(scratch(nA * nB, &s));
    Approx ap;
    CIL_TRY(approx_pass(A, nA, B, nB, dim, &ap, st));
    if (device_radii) {
        CIL_TRY(range_radii_device(A, nA, B, nB, dim, ap, s, M, law, st));
    } else {
        CIL_TRY(range_from_approx(A, nA, B, nB, dim, ap, s, 0, dmin, dmax, st));
        ab->nrange = t_rechecked;
        ab->nrange_exact = t_exact;
        CIL_TRY(radii_ladder(*dmin, *dmax, M, law, radii));
        char *hs;
        CIL_TRY(host_stage(HS_DIST, 4096 + 64, (void **)&hs));
        double *thr = (double *)hs;
        for (int m = 0; m < M; ++m) thr[m] = radii[m] * radii[m];
        CIL_HIP(hipMemcpyAsync(s.thr, thr, sizeof(double) * M, hipMemcpyHostToDevice, st));
    }
    CIL_TRY(fill_zero(s.hist, (char *)(s.nlist + 2) - (char *)s.hist, st));
    ClassifyArgs &c = ap.c;
    c.exclude_diag = 0;
    c.mode = MODE_BINS;
    c.thr = s.thr;
    // With the device's radii, every pair within 2^-44 thr of a threshold is
    // re-checked and its threshold marked: the host's ladder differs from the
    // device's by a few units in the last place at most (where the C
    // library's pow misrounds), so the bins are those of either ladder unless
    // a marked threshold is one where they differ.
    c.thr_slack = device_radii ? 0x1p-44 : 0.0;
    c.M = M;
    c.hist = s.hist;
    c.bins = bins;
    c.list = s.list;
    c.nlist = s.nlist;
    c.cap = s.cap;
    CIL_TRY(classify(c, nA, nB, st));
    CanonOut co{};
    co.pairs = s.list;
    co.npairs_dev = s.nlist;
    co.cap = s.cap;
    co.thr = s.thr;
    co.M = M;
    co.hist = s.hist;
    co.bins = bins;
    co.nB = nB;
    co.nexact = s.nexact;
    co.force_exact = g_force_exact;
    if (device_radii) {
        co.win_rel = 0x1p-44;
        co.win_hits = s.nlist + 7;
    }
    CIL_TRY(canonical_any_length(A, B, dim, co, s.cap, st));
    ab->hist = s.hist;
    ab->nlist = s.nlist;
    ab->cap = s.cap;
    ab->ro = device_radii ? s.ro : nullptr;
    return CIL_OK;
}

template int adaptive_bins_async<double>(const double *, long long, const double *, long long, long long, int, int,
                                         int, double *, double *, double *, uint8_t *, AsyncBins *, hipStream_t);
template int adaptive_bins_async<float>(const float *, long long, const float *, long long, long long, int, int,
                                        int, double *, double *, double *, uint8_t *, AsyncBins *, hipStream_t);

template int adaptive_bins_impl<double>(const double *, long long, const double *, long long, long long, int, int,
                                        int, double *, double *, double *, uint8_t *,
                                        std::vector<unsigned long long> &, hipStream_t);
template int adaptive_bins_impl<float>(const float *, long long, const float *, long long, long long, int, int, int,
                                       double *, double *, double *, uint8_t *, std::vector<unsigned long long> &,
                                       hipStream_t);

template int pair_bins_impl<double>(const double *, long long, const double *, long long, long long, const double *,
                                    int, uint8_t *, std::vector<unsigned long long> &, hipStream_t);
template int pair_bins_impl<float>(const float *, long long, const float *, long long, long long, const double *, int,
                                   uint8_t *, std::vector<unsigned long long> &, hipStream_t);

template <typename T>
int distance_range_impl(const T *A, long long nA, const T *B, long long nB, long long dim, int excl, double *dmin,
                        double *dmax, hipStream_t st)
{
    DistScratch s;
    CIL_TRY(scratch(nA * nB, &s));
    Approx ap;
    CIL_TRY(approx_pass(A, nA, B, nB, dim, &ap, st));
    return range_from_approx(A, nA, B, nB, dim, ap, s, excl, dmin, dmax, st);
}

template int distance_range_impl<double>(const double *, long long, const double *, long long, long long, int,
                                         double *, double *, hipStream_t);
template int distance_range_impl<float>(const float *, long long, const float *, long long, long long, int, double *,
                                        double *, hipStream_t);

// The fast-pass approximation and its bound for every pair (diagnostics).
template <typename T>
int approx_d2_impl(const T *A, long long nA, const T *B, long long nB, long long dim, double *d2, double *eps,
                   hipStream_t st)
{
    Approx ap;
    CIL_TRY(approx_pass(A, nA, B, nB, dim, &ap, st));
    ap.c.mode = MODE_DUMP;
    ap.c.dump_d = d2;
    ap.c.dump_eps = eps;
    CIL_TRY(classify(ap.c, nA, nB, st));
    t_pairs = nA * nB;
    return CIL_OK;
}

template int approx_d2_impl<double>(const double *, long long, const double *, long long, long long, double *,
                                    double *, hipStream_t);
template int approx_d2_impl<float>(const float *, long long, const float *, long long, long long, double *, double *,
                                   hipStream_t);

template <typename T>
int canonical_pairs_impl(const T *A, long long nA, const T *B, long long nB, long long dim, const long long *ia,
                         const long long *jb, long long np, double *d2, hipStream_t st)
{
    DistScratch s;
    CIL_TRY(scratch(1, &s));
    // the list counter slot doubles as the bad-index flag here; nexact counts fallbacks
    CIL_TRY(fill_zero(s.nlist, sizeof(unsigned long long) * 2, st));
    CanonOut co{};
    co.ia = ia;
    co.jb = jb;
    co.npairs = np;
    co.nA = nA;
    co.nB = nB;
    co.bad = (int *)s.nlist;
    co.d2 = d2;
    co.nexact = s.nexact;
    co.force_exact = g_force_exact;
    CIL_TRY(run_canonical(A, B, dim, co, np, st));
    unsigned long long flags[2];
    CIL_HIP(hipMemcpyAsync(flags, s.nlist, sizeof(flags), hipMemcpyDeviceToHost, st));
    CIL_TRY(stream_wait(st));
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
