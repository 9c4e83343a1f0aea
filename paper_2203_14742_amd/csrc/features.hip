// Pattern features beyond the L2 distance (Sec. 3.1 multi-feature CIL, the
// scaled-data experiments of Sec. 5):
//   * min-max scaling of each species of a pattern;
//   * derivative augmentation: a pattern followed by its forward differences
//     along x and y, so that the W^{1,2} norm of a difference is the L2
//     distance of augmented vectors (the split-bf16x3 Gram path serves it);
//   * max-abs distances per segment of a vector (L-infinity of the pattern,
//     of each derivative), their combination by max (W^{1,inf}) or sum (the
//     W^{1,inf} variant with a sum over derivatives), and the binning of such
//     distances under radii.
//
// Values that decide a bin are exact or correctly rounded:
//   * max_k |a_k - b_k| is taken over fl64(|a_k - b_k|); rounding is monotone,
//     so the result is fl64 of the exact maximum;
//   * scaled and augmented values are formed in FP64 with IEEE operations in a
//     fixed order and rounded once to the pattern's type.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cil_internal.hpp"

#pragma clang fp contract(off)

namespace cil {

namespace {

template <typename T>
__device__ __forceinline__ double to64(T v) { return (double)v; }

// ---------------------------------------------------------- min-max scaling
// One workgroup per (pattern, species): s~ = (s - min) / (max - min), in FP64,
// rounded to T; a constant species (max == min) maps to 0.
template <typename T>
__global__ __launch_bounds__(256) void k_minmax_scale(const T *X, long long nn, T *Y)
{
    __shared__ double rmin[4], rmax[4];
    const long long base = ((long long)blockIdx.y * 2 + blockIdx.x) * nn;
    const T *x = X + base;
    T *y = Y + base;
    double lo = INFINITY, hi = -INFINITY;
    for (long long k = threadIdx.x; k < nn; k += 256) {
        const double v = to64(x[k]);
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        rmin[threadIdx.x >> 6] = lo;
        rmax[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    lo = fmin(fmin(rmin[0], rmin[1]), fmin(rmin[2], rmin[3]));
    hi = fmax(fmax(rmax[0], rmax[1]), fmax(rmax[2], rmax[3]));
    const double span = hi - lo;
    for (long long k = threadIdx.x; k < nn; k += 256) {
        const double v = to64(x[k]);
        y[k] = span > 0.0 ? (T)((v - lo) / span) : (T)0.0;
    }
}

// ------------------------------------------------------------ augmentation
// Pattern p ([2][n][n]) -> [s (2 n^2) | D_x s (2 n (n-1)) | D_y s (2 n (n-1))],
// D_x s[c][i][j] = (s[c][i][j+1] - s[c][i][j]) / h, j < n - 1;
// D_y s[c][i][j] = (s[c][i+1][j] - s[c][i][j]) / h, i < n - 1.
template <typename T>
__global__ __launch_bounds__(256) void k_augment(const T *X, int n, double h, long long daug, T *Y)
{
    const long long p = blockIdx.y;
    const long long nn = (long long)n * n, ne = (long long)n * (n - 1);
    const T *x = X + p * 2 * nn;
    T *y = Y + p * daug;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < daug; e += (long long)gridDim.x * 256) {
        if (e < 2 * nn) {
            y[e] = x[e];
        } else if (e < 2 * nn + 2 * ne) {
            const long long f = e - 2 * nn, c = f / ne, r = f % ne, i = r / (n - 1), j = r % (n - 1);
            const long long a = c * nn + i * n + j;
            y[e] = (T)((to64(x[a + 1]) - to64(x[a])) / h);
        } else {
            const long long f = e - 2 * nn - 2 * ne, c = f / ne, r = f % ne, i = r / n, j = r % n;
            const long long a = c * nn + i * n + j;
            y[e] = (T)((to64(x[a + n]) - to64(x[a])) / h);
        }
    }
}

// ------------------------------------------------------- max-abs distances
// One 64 x 64 tile of pairs and one K range [kb, kb + ksplit) per workgroup;
// thread (ty, tx) owns rows ty + 16 i and columns tx + 16 j, i, j < 4.  For
// each segment [e_{s-1}, e_s) the range meets, the tile's partial maxima go
// to out[(i nB + j) nseg + s] by an atomic max on the bit patterns (the values
// are non-negative doubles, whose order is that of their bits), so the
// result is independent of the order of the K ranges; out starts at +0.
constexpr int MT = 64, MKC = 32, MAX_SEG = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_pair_maxabs(const T *A, long long nA, const T *B, long long nB, long long dim,
                                                     const long long *seg_end, int nseg, long long ksplit,
                                                     unsigned long long *out)
{
    __shared__ double sA[MT][MKC + 1];
    __shared__ double sB[MT][MKC + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const long long i0 = (long long)blockIdx.y * MT, j0 = (long long)blockIdx.x * MT;
    const long long kb = (long long)blockIdx.z * ksplit, ke = std::min<long long>(dim, kb + ksplit);
    long long sb = 0;
    for (int s = 0; s < nseg; ++s) {
        const long long se = seg_end[s];
        const long long lo = std::max<long long>(kb, sb), hi = std::min<long long>(ke, se);
        sb = se;
        if (lo >= hi) continue;                     // uniform: this range does not meet segment s
        double m[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) m[a][b] = 0.0;
        for (long long k0 = lo; k0 < hi; k0 += MKC) {
            __syncthreads();
            for (int e = tid; e < MT * MKC; e += 256) {
                const int r = e / MKC, kk = e % MKC;
                const long long k = k0 + kk, ia = i0 + r, jb = j0 + r;
                // positions past the range repeat its first element: |a - b|
                // there is one of the range's own terms, so the max is unchanged
                const long long kc = k < hi ? k : k0;
                sA[r][kk] = ia < nA ? to64(A[ia * dim + kc]) : 0.0;
                sB[r][kk] = jb < nB ? to64(B[jb * dim + kc]) : 0.0;
            }
            __syncthreads();
#pragma unroll 8
            for (int kk = 0; kk < MKC; ++kk) {
                double av[4], bv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = sA[ty + 16 * a][kk];
#pragma unroll
                for (int b = 0; b < 4; ++b) bv[b] = sB[tx + 16 * b][kk];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) m[a][b] = fmax(m[a][b], fabs(av[a] - bv[b]));
            }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const long long i = i0 + ty + 16 * a, j = j0 + tx + 16 * b;
                if (i < nA && j < nB && m[a][b] > 0.0)
                    atomicMax(&out[(i * nB + j) * nseg + s], (unsigned long long)__double_as_longlong(m[a][b]));
            }
    }
}

// out[p] over D[p][0..nseg-1]: mode 0 max, 1 left-to-right sum, 2 left-to-right
// sum of the (correctly rounded) square roots
__global__ void k_combine(const double *D, long long n, int nseg, int mode, double *out)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double *d = D + p * nseg;
    double v = mode == 2 ? sqrt(d[0]) : d[0];
    for (int s = 1; s < nseg; ++s) v = mode == 0 ? fmax(v, d[s]) : v + (mode == 2 ? sqrt(d[s]) : d[s]);
    out[p] = v;
}

// min and max of V (as ordered bit patterns of non-negative doubles)
__global__ __launch_bounds__(256) void k_value_range(const double *V, long long n, unsigned long long *mm)
{
    __shared__ unsigned long long rlo[4], rhi[4];
    unsigned long long lo = ~0ull, hi = 0ull;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const unsigned long long b = __double_as_longlong(V[p]);
        lo = b < lo ? b : lo;
        hi = b > hi ? b : hi;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long l2 = __shfl_xor(lo, o, 64), h2 = __shfl_xor(hi, o, 64);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    if ((threadIdx.x & 63) == 0) {
        rlo[threadIdx.x >> 6] = lo;
        rhi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            lo = rlo[w] < lo ? rlo[w] : lo;
            hi = rhi[w] > hi ? rhi[w] : hi;
        }
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
    }
}

// bins[p] = #{m : V[p] < radii[m]} (radii decreasing), hist[b] += 1
constexpr int VMAX_M = 255;
__global__ __launch_bounds__(256) void k_bin_values(const double *V, long long n, const double *radii, int M,
                                                    uint8_t *bins, unsigned long long *hist)
{
    __shared__ double r[VMAX_M];
    __shared__ unsigned int h[VMAX_M + 1];
    for (int m = threadIdx.x; m < M; m += 256) r[m] = radii[m];
    for (int m = threadIdx.x; m <= M; m += 256) h[m] = 0;
    __syncthreads();
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const double v = V[p];
        int c = 0;
        while (c < M && v < r[c]) ++c;
        if (bins) bins[p] = (uint8_t)c;
        atomicAdd(&h[c], 1u);
    }
    __syncthreads();
    for (int m = threadIdx.x; m <= M; m += 256)
        if (h[m]) atomicAdd(&hist[m], (unsigned long long)h[m]);
}

unsigned grid_for(long long n, long long cap = 4096)
{
    return (unsigned)std::max<long long>(1, std::min<long long>(cap, (n + 255) / 256));
}

}  // namespace

int minmax_scale_impl(const void *X, long long count, int n, cil_precision prec, void *Y, hipStream_t st)
{
    if (count == 0) return CIL_OK;
    const long long nn = (long long)n * n;
    dim3 grid(2, (unsigned)count);
    if (prec == CIL_FP32)
        hipLaunchKernelGGL(k_minmax_scale<float>, grid, dim3(256), 0, st, (const float *)X, nn, (float *)Y);
    else
        hipLaunchKernelGGL(k_minmax_scale<double>, grid, dim3(256), 0, st, (const double *)X, nn, (double *)Y);
    return check_launch("k_minmax_scale");
}

int augment_impl(const void *X, long long count, int n, double L, cil_precision prec, void *Y, hipStream_t st)
{
    if (count == 0) return CIL_OK;
    const long long daug = 2ll * n * n + 4ll * n * (n - 1);
    const double h = L / (double)(n - 1);
    dim3 grid((unsigned)std::min<long long>(64, (daug + 255) / 256), (unsigned)count);
    if (prec == CIL_FP32)
        hipLaunchKernelGGL(k_augment<float>, grid, dim3(256), 0, st, (const float *)X, n, h, daug, (float *)Y);
    else
        hipLaunchKernelGGL(k_augment<double>, grid, dim3(256), 0, st, (const double *)X, n, h, daug, (double *)Y);
    return check_launch("k_augment");
}

int pair_maxabs_impl(const void *A, long long nA, const void *B, long long nB, long long dim, cil_precision prec,
                     const int64_t *seg_end, int nseg, double *D, hipStream_t st)
{
    if (nseg < 1 || nseg > MAX_SEG) return set_error(CIL_EINVAL, "nseg must be in [1, %d]", MAX_SEG);
    long long prev = 0;
    for (int s = 0; s < nseg; ++s) {
        if (seg_end[s] < prev || seg_end[s] > dim) return set_error(CIL_EINVAL, "segment ends must rise to <= dim");
        prev = seg_end[s];
    }
    if (nA * nB == 0) return CIL_OK;
    void *p;
    CIL_TRY(ws_get(WS_FEAT_SEG, sizeof(long long) * MAX_SEG, &p));
    long long *dseg = (long long *)p;
    CIL_HIP(hipMemcpyAsync(dseg, seg_end, sizeof(long long) * nseg, hipMemcpyHostToDevice, st));
    CIL_TRY(fill_zero(D, sizeof(double) * (size_t)(nA * nB * nseg), st));
    if (dim == 0) return CIL_OK;
    // split K so that the grid holds about 1024 workgroups
    const long long tiles = ((nA + MT - 1) / MT) * ((nB + MT - 1) / MT), chunks = (dim + MKC - 1) / MKC;
    const long long splits = std::max<long long>(1, std::min<long long>(chunks, (1024 + tiles - 1) / tiles));
    const long long ks = (chunks + splits - 1) / splits * MKC;
    dim3 grid((unsigned)((nB + MT - 1) / MT), (unsigned)((nA + MT - 1) / MT), (unsigned)((dim + ks - 1) / ks));
    unsigned long long *out = (unsigned long long *)D;
    const ProfMark pm = prof_begin("k_pair_maxabs", st);
    if (prec == CIL_FP32)
        hipLaunchKernelGGL(k_pair_maxabs<float>, grid, dim3(256), 0, st, (const float *)A, nA, (const float *)B, nB,
                           dim, (const long long *)dseg, nseg, ks, out);
    else
        hipLaunchKernelGGL(k_pair_maxabs<double>, grid, dim3(256), 0, st, (const double *)A, nA, (const double *)B, nB,
                           dim, (const long long *)dseg, nseg, ks, out);
    prof_end(pm, st);
    return check_launch("k_pair_maxabs");
}

int combine_segments_impl(const double *D, long long n, int nseg, int mode, double *out, hipStream_t st)
{
    if (n == 0) return CIL_OK;
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D, n, nseg, mode, out);
    return check_launch("k_combine");
}

int value_range_impl(const double *V, long long n, double *vmin, double *vmax, hipStream_t st)
{
    void *p;
    CIL_TRY(ws_get(WS_FEAT_MISC, 2 * sizeof(unsigned long long), &p));
    unsigned long long *mm = (unsigned long long *)p;
    const unsigned long long init[2] = {~0ull, 0ull};
    CIL_HIP(hipMemcpyAsync(mm, init, sizeof(init), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_value_range, dim3(grid_for(n)), dim3(256), 0, st, V, n, mm);
    CIL_TRY(check_launch("k_value_range"));
    unsigned long long h[2];
    CIL_HIP(hipMemcpyAsync(h, mm, sizeof(h), hipMemcpyDeviceToHost, st));
    CIL_TRY(stream_wait(st));
    double lo, hi;
    std::memcpy(&lo, &h[0], 8);
    std::memcpy(&hi, &h[1], 8);
    *vmin = lo;
    *vmax = hi;
    return CIL_OK;
}

int bin_values_impl(const double *V, long long n, const double *radii, int M, uint8_t *bins, int64_t *counts,
                    hipStream_t st)
{
    if (M < 1 || M > VMAX_M) return set_error(CIL_EINVAL, "M must be in [1, %d]", VMAX_M);
    void *p;
    CIL_TRY(ws_get(WS_FEAT_MISC, sizeof(unsigned long long) * (M + 1) + sizeof(double) * M, &p));
    unsigned long long *hist = (unsigned long long *)p;
    double *dr = (double *)(hist + M + 1);
    CIL_TRY(fill_zero(hist, sizeof(unsigned long long) * (M + 1), st));
    CIL_HIP(hipMemcpyAsync(dr, radii, sizeof(double) * M, hipMemcpyHostToDevice, st));
    if (n > 0) {
        hipLaunchKernelGGL(k_bin_values, dim3(grid_for(n)), dim3(256), 0, st, V, n, dr, M, bins, hist);
        CIL_TRY(check_launch("k_bin_values"));
    }
    std::vector<unsigned long long> h(M + 1);
    CIL_HIP(hipMemcpyAsync(h.data(), hist, sizeof(unsigned long long) * (M + 1), hipMemcpyDeviceToHost, st));
    CIL_TRY(stream_wait(st));
    unsigned long long tail = 0;
    for (int m = M; m >= 1; --m) {
        tail += h[m];
        counts[m - 1] = (int64_t)tail;
    }
    return CIL_OK;
}

}  // namespace cil
