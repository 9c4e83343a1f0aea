// Split-bf16x3 Gram on the gfx950 matrix cores, for FP32 pattern sets.
//
// Squared distances through the Gram: D(a, b) = |a|^2 + |b|^2 - 2 <a, b>.
// Both sets are first shifted by one common vector c (a sampled column mean,
// which does not change any distance) and each shifted value x' = fl32(x - c)
// is split into two bf16 numbers x' ~ hi + lo (hi = bf16(x'), lo =
// bf16(x' - hi)).  The Gram of the split vectors is taken as three bf16
// products hi.hi + hi.lo + lo.hi on v_mfma_f32_32x32x16_bf16 (products exact,
// FP32 accumulation), promoted to an FP64 accumulator every KC elements
// (64, 128 or 256; CIL_OPT_GRAM_FLUSH).  |a^|^2 is summed in FP64 from (hi + lo).
//
// Error bound (per pair, relative to S = |a'| + |b'| and |a'| |b'|):
//   Gram:     |G~ - <a^, b^>| <= eG = (3 KC 2^-24 + 2^-18 + 2^-40) |a'||b'|
//             (FP32 roundings of the accumulation; the dropped lo.lo term)
//   split:    a^ = (a - c) + e_a with |e_a,k| <= e1 |a'_k|, e1 = 2^-24 + 2^-18
//   distance: |D~ - D| <= 2 eG + 2 e1 S (sqrt(D~+ + 2 eG) + e1 S) + e1^2 S^2
//             + 8 u64 (|a^|^2 + |b^|^2 + D~+) + u64 D
// and the band used is twice that.  Pairs within the band of a threshold are
// recomputed canonically (distance.hip), so counts stay exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "cil_internal.hpp"

namespace cil {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int GT = 128;          // tile side (pairs) per workgroup
constexpr int GK = 64;           // k per LDS stage
constexpr int GPAD = 8;          // row padding (elements) of LDS tiles
constexpr int GKC = 256;         // split-K granularity (elements)

// ------------------------------------------------------------------ shift
// c_k = mean over up to 64 sampled rows of A and B (FP64 sum, rounded to FP32)
// The sampled row offsets (r nA / sa) dim are the same for every thread: the
// first 64 threads of a block compute them once into LDS.
__global__ __launch_bounds__(64) void k_shift_vector(const float *A, long long nA, const float *B, long long nB,
                                                      long long dim, float *c)
{
    __shared__ long long rowoff[64];
    const long long sa = std::min<long long>(nA, 32), sb = std::min<long long>(nB, 32);
    const int t = threadIdx.x;
    if (t < 32) rowoff[t] = t < sa ? (t * nA / sa) * dim : 0;
    else rowoff[t] = t - 32 < sb ? ((t - 32) * nB / sb) * dim : 0;
    __syncthreads();
    const long long k = (long long)blockIdx.x * blockDim.x + t;
    if (k >= dim || sa == 0 || sb == 0) {           // (an empty set: the mean of the other one)
        if (k < dim && (sa | sb)) {
            const float *X = sa ? A : B;
            const long long sx = sa ? sa : sb, nx = sa ? nA : nB;
            double s = 0.0;
            for (long long r = 0; r < sx; ++r) s += X[(r * nx / sx) * dim + k];
            c[k] = (float)(s / (double)sx);
        } else if (k < dim) {
            c[k] = 0.0f;
        }
        return;
    }
    // all sampled values are loaded first (independent, unconditional loads
    // in flight together: rows past the sample repeat row 0 and are not
    // added), then summed in row order
    float va[32], vb[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) {
        va[r] = A[rowoff[r] + k];
        vb[r] = B[rowoff[32 + r] + k];
    }
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 32; ++r)
        if (r < sa) s += va[r];
#pragma unroll
    for (int r = 0; r < 32; ++r)
        if (r < sb) s += vb[r];
    const long long cnt = sa + sb;
    c[k] = cnt ? (float)(s / (double)cnt) : 0.0f;
}

// ------------------------------------------------------------------ split
// One workgroup per row: hi/lo into [n][dimP] (zero padded), |x^|^2 in FP64.
// Rows whose FP32 data (and the shift vector) are 16-byte aligned with
// dim % 4 == 0 move four elements per lane (16-byte loads, 8-byte stores);
// other rows go one element per lane.  The split of each element is the same
// either way; only the order of the FP64 norm accumulation differs.
__device__ __forceinline__ void split_one(float xs, __bf16 &bh, __bf16 &bl, double &s)
{
    bh = (__bf16)xs;
    bl = (__bf16)(xs - (float)bh);
    const double v = (double)(float)bh + (double)(float)bl;
    s = fma(v, v, s);
}

// Both sets in one launch: blocks [0, nX) take rows of X, the rest rows of Y.
__global__ __launch_bounds__(256) void k_split_rows(const float *X, long long nX, __bf16 *hiX, __bf16 *loX,
                                                    double *normX, const float *Y, __bf16 *hiY, __bf16 *loY,
                                                    double *normY, long long dim, long long dimP, const float *c)
{
    __shared__ double red[4];
    const bool first = (long long)blockIdx.x < nX;
    const long long r = first ? (long long)blockIdx.x : (long long)blockIdx.x - nX;
    const float *x = (first ? X : Y) + r * dim;
    __bf16 *h = (first ? hiX : hiY) + r * dimP;
    __bf16 *l = (first ? loX : loY) + r * dimP;
    double *norm2 = first ? normX : normY;
    double s = 0.0;
    const bool vec = (dim & 3) == 0 && (dimP & 3) == 0 && (((uintptr_t)x | (uintptr_t)c) & 15) == 0;
    if (vec) {
#pragma unroll 4
        for (long long k = 4 * (long long)threadIdx.x; k < dimP; k += 4 * (long long)blockDim.x) {
            union {
                __bf16 b[4];
                uint2 u;
            } ph, pl;
            if (k < dim) {                          // dim % 4 == 0: all four elements are data
                const float4 xv = *(const float4 *)(x + k);
                const float4 cv = *(const float4 *)(c + k);
                split_one(xv.x - cv.x, ph.b[0], pl.b[0], s);
                split_one(xv.y - cv.y, ph.b[1], pl.b[1], s);
                split_one(xv.z - cv.z, ph.b[2], pl.b[2], s);
                split_one(xv.w - cv.w, ph.b[3], pl.b[3], s);
            } else {
                ph.u = make_uint2(0u, 0u);
                pl.u = make_uint2(0u, 0u);
            }
            *(uint2 *)(h + k) = ph.u;
            *(uint2 *)(l + k) = pl.u;
        }
    } else {
        for (long long k = threadIdx.x; k < dimP; k += blockDim.x) {
            __bf16 bh = (__bf16)0.0f, bl = (__bf16)0.0f;
            if (k < dim) split_one(x[k] - c[k], bh, bl, s);
            h[k] = bh;
            l[k] = bl;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) norm2[r] = red[0] + red[1] + red[2] + red[3];
}

// ------------------------------------------------------------------ Gram
// Grid (tiles over B, tiles over A, K splits).  Four wavefronts, each a 64 x 64
// block of the 128 x 128 tile as 2 x 2 MFMA 32 x 32 tiles.  Output: FP64
// partial Gram P[split][i][j].  Registers are held to 256 so that two
// workgroups share a CU (LDS 2 x 74 KB): one stages its next tiles while the
// other runs its MFMAs.
//
// v_mfma_f32_32x32x16_bf16 lane layout: lane l supplies row l%32 of the A
// block and row l%32 of the B block (a column of B^T), elements
// k = 8 (l/32) .. 8 (l/32) + 7 of the 16-wide k step; accumulator element r of
// lane l is C[8 (r/4) + 4 (l/32) + r%4][l%32].
template <int KCF>   // FP32 -> FP64 promotion interval (elements), a multiple of GK
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gram_bf16x3(const __bf16 *Ah, const __bf16 *Al, long long nA,
                                                     const __bf16 *Bh, const __bf16 *Bl, long long nB,
                                                     long long dimP, long long ksplit, double *P)
{
    __shared__ __attribute__((aligned(16))) __bf16 sAh[GT][GK + GPAD];
    __shared__ __attribute__((aligned(16))) __bf16 sAl[GT][GK + GPAD];
    __shared__ __attribute__((aligned(16))) __bf16 sBh[GT][GK + GPAD];
    __shared__ __attribute__((aligned(16))) __bf16 sBl[GT][GK + GPAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int wr = wv >> 1, wc = wv & 1;
    const long long i0 = (long long)blockIdx.y * GT, j0 = (long long)blockIdx.x * GT;
    const long long kb = (long long)blockIdx.z * ksplit;
    const long long ke = std::min<long long>(dimP, kb + ksplit);

    floatx16 acc[2][2];
    double acc64[2][2][16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc[a][b][r] = 0.0f;
                acc64[a][b][r] = 0.0;
            }
        }

    int since_flush = 0;
    for (long long k0 = kb; k0 < ke; k0 += GK) {
        __syncthreads();
        // stage 128 rows x 64 k of each split array: 16-byte chunks, 8 per row
        for (int e = tid; e < GT * (GK / 8); e += 256) {
            const int row = e / (GK / 8), ch = e % (GK / 8);
            const long long ia = i0 + row, jb = j0 + row;
            const long long off = k0 + 8 * ch;
            bf16x8 z;
#pragma unroll
            for (int t = 0; t < 8; ++t) z[t] = (__bf16)0.0f;
            const bool ka = off < ke;
            *(bf16x8 *)&sAh[row][8 * ch] = (ia < nA && ka) ? *(const bf16x8 *)(Ah + ia * dimP + off) : z;
            *(bf16x8 *)&sAl[row][8 * ch] = (ia < nA && ka) ? *(const bf16x8 *)(Al + ia * dimP + off) : z;
            *(bf16x8 *)&sBh[row][8 * ch] = (jb < nB && ka) ? *(const bf16x8 *)(Bh + jb * dimP + off) : z;
            *(bf16x8 *)&sBl[row][8 * ch] = (jb < nB && ka) ? *(const bf16x8 *)(Bl + jb * dimP + off) : z;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            const int kofs = kk + 8 * (lane >> 5);
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ra = wr * 64 + t * 32 + (lane & 31);
                const int rb = wc * 64 + t * 32 + (lane & 31);
                ah[t] = *(const bf16x8 *)&sAh[ra][kofs];
                al[t] = *(const bf16x8 *)&sAl[ra][kofs];
                bh[t] = *(const bf16x8 *)&sBh[rb][kofs];
                bl[t] = *(const bf16x8 *)&sBl[rb][kofs];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                }
        }
        since_flush += GK;
        if (since_flush >= KCF) {
            since_flush = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        acc64[a][b][r] += (double)acc[a][b][r];
                        acc[a][b][r] = 0.0f;
                    }
        }
    }
    double *Ps = P + (long long)blockIdx.z * nA * nB;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const long long i = i0 + wr * 64 + a * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
                const long long j = j0 + wc * 64 + b * 32 + (lane & 31);
                if (i < nA && j < nB) Ps[i * nB + j] = acc64[a][b][r] + (double)acc[a][b][r];
            }
}

// Pipelined variant (the default).  Tiles are staged by LDS-DMA loads
// (global_load_lds_dwordx4: the 16 bytes of lane l land at the wave's LDS base
// + 16 l, no registers) into two LDS buffers of GD = 32 k: the loads of stage
// s + 1 are in flight while the matrix cores work on stage s, one barrier per
// stage.  Wavefront w stages array w (A hi, A lo, B hi, B lo) in 8
// instructions of 64 slots.  The 16-byte chunk c of tile row r sits in slot
// 4 r + (c ^ swz(r)): the fragment reads (32 consecutive rows, one chunk per
// half-wave) then fall on distinct banks for 32- and 64-bank LDS alike.  Rows
// past the end of a set load the last row (their sums are never stored).  Same
// products, order and promotion points as k_gram_bf16x3, so the two give
// identical sums.  Measured on 2048 x 2048 x 32768: 1.04 ms (0.79 PFLOP/s
// executed bf16) against 1.69 ms for k_gram_bf16x3; deeper pipelines of
// 16-k stages (4 or 5 buffers) were slower (1.7-1.8 ms).
//
// With `xcd_order`, consecutive tiles of the (j, i, split) order are given to
// one XCD (workgroups reach the 8 XCDs round-robin in launch order), so an XCD
// works on whole rows of tiles and its L2 holds the A rows they share
// (1.03 against 1.07 ms).
constexpr int GD = 32;

__device__ __forceinline__ int gram_swz(int r) { return (((r >> 1) ^ (r >> 3)) & 1) | (((r >> 2) & 1) << 1); }

template <int KCF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gram_dma(
    const __bf16 *Ah, const __bf16 *Al, long long nA, const __bf16 *Bh, const __bf16 *Bl, long long nB,
    long long dimP, long long ksplit, double *P, int xcd_order)
{
    constexpr int CPR = GD / 8;                  // 16-byte chunks per tile row per stage
    constexpr int PARTS = GT * CPR / 64;         // DMA instructions per wavefront per stage
    __shared__ __attribute__((aligned(16))) uint4 sm[2][4][GT * CPR];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wv >> 1, wc = wv & 1;
    long long tx = blockIdx.x, ty = blockIdx.y, tz = blockIdx.z;
    if (xcd_order) {
        const long long gx = gridDim.x, gy = gridDim.y, tot = gx * gy * gridDim.z;
        const long long L = tx + gx * (ty + gy * tz);
        const long long per = tot / 8;
        if (L < per * 8) {                       // full rounds of 8: XCD L % 8 takes a contiguous range
            const long long Lp = (L % 8) * per + L / 8;
            tx = Lp % gx;
            ty = (Lp / gx) % gy;
            tz = Lp / (gx * gy);
        }
    }
    const long long i0 = ty * GT, j0 = tx * GT;
    const long long kb = tz * ksplit;
    const long long ke = std::min<long long>(dimP, kb + ksplit);

    const __bf16 *src = wv == 0 ? Ah : (wv == 1 ? Al : (wv == 2 ? Bh : Bl));
    const long long r0 = wv < 2 ? i0 : j0;
    const long long nr = wv < 2 ? nA : nB;
    const int drow = lane / CPR;                                   // row of slot 64 p + lane, minus 64 p / CPR
    const int dchunk = (lane % CPR) ^ gram_swz(drow);
    auto stage = [&](long long k0, int b) {
#pragma unroll
        for (int p = 0; p < PARTS; ++p) {
            const long long row = std::min<long long>(r0 + (64 / CPR) * p + drow, nr - 1);
            const __bf16 *g = src + row * dimP + k0 + 8 * dchunk;
            __builtin_amdgcn_global_load_lds((const void *)g,
                                             (__attribute__((address_space(3))) void *)&sm[b][wv][64 * p], 16, 0, 0);
        }
    };

    floatx16 acc[2][2];
    double acc64[2][2][16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc[a][b][r] = 0.0f;
                acc64[a][b][r] = 0.0;
            }
        }

    const int fsw = gram_swz(lane & 31);
    stage(kb, 0);
    int buf = 0, since_flush = 0;
    for (long long k0 = kb; k0 < ke; k0 += GD) {
        // this wavefront's loads of stage k0 have landed (vmcnt(0); gfx9
        // s_waitcnt: vmcnt 3:0 and 15:14, expcnt 6:4 = 7 and lgkmcnt 11:8 = 15
        // mean no wait on those)
        __builtin_amdgcn_s_waitcnt(0x0F70);
        // Bare workgroup barrier: a __syncthreads fence would also wait for
        // every outstanding DMA load (vmcnt(0)) and drain the prefetch.  The
        // loop writes LDS only by DMA (covered by the wait above) and every
        // LDS read of the buffer refilled next was consumed (lgkmcnt waited)
        // in the previous iteration; the asm clobber keeps the compiler from
        // moving LDS accesses across the barrier.
        asm volatile("s_barrier" ::: "memory");
        if (k0 + GD < ke) stage(k0 + GD, buf ^ 1);
        const uint4 *sAh = sm[buf][0], *sAl = sm[buf][1], *sBh = sm[buf][2], *sBl = sm[buf][3];
#pragma unroll
        for (int kk = 0; kk < GD; kk += 16) {
            const int c = (kk >> 3) + (lane >> 5);
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ra = wr * 64 + t * 32 + (lane & 31);
                const int rb = wc * 64 + t * 32 + (lane & 31);
                ah[t] = __builtin_bit_cast(bf16x8, sAh[CPR * ra + (c ^ fsw)]);
                al[t] = __builtin_bit_cast(bf16x8, sAl[CPR * ra + (c ^ fsw)]);
                bh[t] = __builtin_bit_cast(bf16x8, sBh[CPR * rb + (c ^ fsw)]);
                bl[t] = __builtin_bit_cast(bf16x8, sBl[CPR * rb + (c ^ fsw)]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                }
        }
        buf ^= 1;
        since_flush += GD;
        if (since_flush >= KCF) {
            since_flush = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        acc64[a][b][r] += (double)acc[a][b][r];
                        acc[a][b][r] = 0.0f;
                    }
        }
    }
    double *Ps = P + tz * nA * nB;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const long long i = i0 + wr * 64 + a * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
                const long long j = j0 + wc * 64 + b * 32 + (lane & 31);
                if (i < nA && j < nB) Ps[i * nB + j] = acc64[a][b][r] + (double)acc[a][b][r];
            }
}

// ---------------------------------------------------------------- host
struct GramWork {
    __bf16 *Ah, *Al, *Bh, *Bl;
    double *na, *nb;
    float *c;
    long long dimP;
};

int gram_prepare(const float *A, long long nA, const float *B, long long nB, long long dim, GramWork *g,
                 hipStream_t st)
{
    const long long dimP = std::max<long long>(GK, (dim + GK - 1) / GK * GK);
    void *p;
    const size_t sa = sizeof(__bf16) * (size_t)std::max<long long>(nA, 1) * dimP;
    const size_t sb = sizeof(__bf16) * (size_t)std::max<long long>(nB, 1) * dimP;
    CIL_TRY(ws_get(WS_DIST_SPLIT_A, 2 * sa, &p));
    g->Ah = (__bf16 *)p;
    g->Al = (__bf16 *)((char *)p + sa);
    CIL_TRY(ws_get(WS_DIST_SPLIT_B, 2 * sb, &p));
    g->Bh = (__bf16 *)p;
    g->Bl = (__bf16 *)((char *)p + sb);
    CIL_TRY(ws_get(WS_DIST_COUNTS, sizeof(double) * (size_t)(nA + nB + 2) + sizeof(float) * (size_t)dimP + 64, &p));
    g->na = (double *)p;
    g->nb = g->na + nA + 1;
    g->c = (float *)(((uintptr_t)(g->nb + nB + 1) + 15) & ~(uintptr_t)15);   // 16-byte aligned (64 B of slack)
    g->dimP = dimP;
    if (dim > 0) {
        const ProfMark pm = prof_begin("k_shift_vector", st);
        hipLaunchKernelGGL(k_shift_vector, dim3((unsigned)((dim + 63) / 64)), dim3(64), 0, st, A, nA, B, nB, dim, g->c);
        prof_end(pm, st);
        CIL_TRY(check_launch("k_shift_vector"));
    }
    const ProfMark pm = prof_begin("k_split_rows", st);
    if (nA + nB > 0)
        hipLaunchKernelGGL(k_split_rows, dim3((unsigned)(nA + nB)), dim3(256), 0, st, A, nA, g->Ah, g->Al, g->na, B,
                           g->Bh, g->Bl, g->nb, dim, dimP, (const float *)g->c);
    prof_end(pm, st);
    return check_launch("k_split_rows");
}

// FP32 -> FP64 promotion interval of the Gram (64, 128 or 256 elements; 64:
// the narrowest band, fewest re-checks, no measurable cost in the Gram); the
// classification's error bound uses the same value.
int g_gram_kc = 64;
// 0: k_gram_bf16x3; 1: k_gram_dma in launch order; 2: k_gram_dma in XCD order
int g_gram_pipeline = 2;
int set_gram_pipeline(int64_t v)
{
    if (v < 0 || v > 2) return set_error(CIL_EINVAL, "Gram pipeline option %lld not in {0, 1, 2}", (long long)v);
    g_gram_pipeline = (int)v;
    return CIL_OK;
}
// effective interval: the register-staged kernel promotes at multiples of its 64-k stage
int gram_flush_interval() { return g_gram_pipeline ? g_gram_kc : std::max(g_gram_kc, GK); }
int set_gram_flush_interval(int64_t v)
{
    if (v != 32 && v != 64 && v != 128 && v != 256)
        return set_error(CIL_EINVAL, "Gram flush interval %lld not in {32, 64, 128, 256}", (long long)v);
    g_gram_kc = (int)v;
    return CIL_OK;
}

// number of K splits so that the grid holds enough workgroups
long long gram_splits(long long nA, long long nB, long long dimP)
{
    const long long tiles = ((nA + GT - 1) / GT) * ((nB + GT - 1) / GT);
    long long s = 1;
    while (tiles * s < 1024 && (dimP / (s * 2)) >= GKC) s *= 2;
    return s;
}

// splits x ks must cover dimP; ks a multiple of GK
int gram_partials(const GramWork &g, long long nA, long long nB, long long splits, long long ks, double *P,
                  hipStream_t st)
{
    if (ks % GK != 0 || splits * ks < g.dimP) return set_error(CIL_EINVAL, "bad Gram split");
    dim3 grid((unsigned)((nB + GT - 1) / GT), (unsigned)((nA + GT - 1) / GT), (unsigned)splits);
    const int kc = gram_flush_interval();
    if (g_gram_pipeline) {
        const ProfMark pm2 = prof_begin("k_gram_dma", st);
        const __bf16 *ah = g.Ah, *al = g.Al, *bh = g.Bh, *bl = g.Bl;
        const int xo = g_gram_pipeline == 2;
        if (kc == 32)
            hipLaunchKernelGGL(k_gram_dma<32>, grid, dim3(256), 0, st, ah, al, nA, bh, bl, nB, g.dimP, ks, P, xo);
        else if (kc == 64)
            hipLaunchKernelGGL(k_gram_dma<64>, grid, dim3(256), 0, st, ah, al, nA, bh, bl, nB, g.dimP, ks, P, xo);
        else if (kc == 128)
            hipLaunchKernelGGL(k_gram_dma<128>, grid, dim3(256), 0, st, ah, al, nA, bh, bl, nB, g.dimP, ks, P, xo);
        else
            hipLaunchKernelGGL(k_gram_dma<256>, grid, dim3(256), 0, st, ah, al, nA, bh, bl, nB, g.dimP, ks, P, xo);
        prof_end(pm2, st);
        return check_launch("k_gram_dma");
    }
    const ProfMark pm = prof_begin("k_gram_bf16x3", st);
    if (kc <= 64)
        hipLaunchKernelGGL(k_gram_bf16x3<64>, grid, dim3(256), 0, st, (const __bf16 *)g.Ah, (const __bf16 *)g.Al, nA,
                           (const __bf16 *)g.Bh, (const __bf16 *)g.Bl, nB, g.dimP, ks, P);
    else if (kc == 128)
        hipLaunchKernelGGL(k_gram_bf16x3<128>, grid, dim3(256), 0, st, (const __bf16 *)g.Ah, (const __bf16 *)g.Al,
                           nA, (const __bf16 *)g.Bh, (const __bf16 *)g.Bl, nB, g.dimP, ks, P);
    else
        hipLaunchKernelGGL(k_gram_bf16x3<256>, grid, dim3(256), 0, st, (const __bf16 *)g.Ah, (const __bf16 *)g.Al,
                           nA, (const __bf16 *)g.Bh, (const __bf16 *)g.Bl, nB, g.dimP, ks, P);
    prof_end(pm, st);
    return check_launch("k_gram_bf16x3");
}

}  // namespace cil
