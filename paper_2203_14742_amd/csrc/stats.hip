// Bootstrap correlation integral vectors (Alg. 2bst / Alg. 3bst step 2) and
// the Gaussian synthetic likelihood (eqs. cil:CF, cil:CF_synth) on gfx950.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

#include "cil_internal.hpp"

namespace cil {

// ------------------------------------------------------------- bootstrap
// One workgroup per (resample, slice of its kA rows).  For every selected
// pair the byte bins[i][j] (number of radii the pair is under) is compared
// against m = 0..MAXM-1 and accumulated in per-lane counters:
// count[m] += (bin > m).  Counters are reduced over the workgroup and added
// to Ycount with 64-bit atomics.
template <int MAXM>
__global__ __launch_bounds__(256) void k_bootstrap(const uint8_t *bins, long long nA, long long nB, int M,
                                                   const int *idxA, int kA, const int *idxB, int kB,
                                                   int rows_per_block, unsigned long long *Ycnt,
                                                   int *bad, const int *only_if)
{
    if (only_if && !(only_if[1] && !only_if[0])) return;   // after the MFMA path: only if it declined
    extern __shared__ int sh[];
    int *sidx = sh;                          // kB column indices of this resample
    unsigned int *red = (unsigned int *)(sh + kB);
    const int r = blockIdx.y;
    const int tid = threadIdx.x;
    for (int b = tid; b < kB; b += blockDim.x) {
        int j = idxB[(long long)r * kB + b];
        if (j < 0 || j >= nB) {
            atomicOr(bad, 1);
            j = 0;
        }
        sidx[b] = j;
    }
    for (int m = tid; m < MAXM; m += blockDim.x) red[m] = 0;
    __syncthreads();
    unsigned int cnt[MAXM];
#pragma unroll
    for (int m = 0; m < MAXM; ++m) cnt[m] = 0;
    const int a0 = blockIdx.x * rows_per_block;
    const int a1 = min(kA, a0 + rows_per_block);
    for (int a = a0; a < a1; ++a) {
        long long i = idxA[(long long)r * kA + a];
        if (i < 0 || i >= nA) {
            atomicOr(bad, 1);
            continue;
        }
        const uint8_t *row = bins + i * nB;
        for (int b = tid; b < kB; b += blockDim.x) {
            const int v = row[sidx[b]];
#pragma unroll
            for (int m = 0; m < MAXM; ++m) cnt[m] += (v > m);
        }
    }
#pragma unroll
    for (int m = 0; m < MAXM; ++m) {
        unsigned int c = cnt[m];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if ((tid & 63) == 0 && m < M && c) atomicAdd(&red[m], c);
    }
    __syncthreads();
    for (int m = tid; m < M; m += blockDim.x)
        if (red[m]) atomicAdd(&Ycnt[(long long)r * M + m], (unsigned long long)red[m]);
}

// Large M (> 64): a per-block LDS histogram of the bin values, then suffix
// sums: #{bin > m} = sum over v > m of hist[v].
__global__ __launch_bounds__(256) void k_bootstrap_hist(const uint8_t *bins, long long nA, long long nB, int M,
                                                        const int *idxA, int kA, const int *idxB, int kB,
                                                        int rows_per_block, unsigned long long *Ycnt, int *bad,
                                                        const int *only_if)
{
    if (only_if && !(only_if[1] && !only_if[0])) return;
    extern __shared__ int sh[];
    int *sidx = sh;
    unsigned int *hist = (unsigned int *)(sh + kB);
    const int r = blockIdx.y;
    const int tid = threadIdx.x;
    for (int b = tid; b < kB; b += blockDim.x) {
        int j = idxB[(long long)r * kB + b];
        if (j < 0 || j >= nB) {
            atomicOr(bad, 1);
            j = 0;
        }
        sidx[b] = j;
    }
    for (int m = tid; m < 256; m += blockDim.x) hist[m] = 0;
    __syncthreads();
    const int a0 = blockIdx.x * rows_per_block;
    const int a1 = min(kA, a0 + rows_per_block);
    for (int a = a0; a < a1; ++a) {
        long long i = idxA[(long long)r * kA + a];
        if (i < 0 || i >= nA) {
            atomicOr(bad, 1);
            continue;
        }
        const uint8_t *row = bins + i * nB;
        for (int b = tid; b < kB; b += blockDim.x) atomicAdd(&hist[row[sidx[b]]], 1u);
    }
    __syncthreads();
    if (tid < M) {
        unsigned long long c = 0;
        for (int v = tid + 1; v < 256; ++v) c += hist[v];
        if (c) atomicAdd(&Ycnt[(long long)r * M + tid], c);
    }
}

__global__ void k_boot_finish(const unsigned long long *Ycnt, long long n, double denom, long long *Yc,
                              double *Y)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const unsigned long long c = Ycnt[e];
    if (Yc) Yc[e] = (long long)c;
    if (Y) Y[e] = (double)c / denom;
}

// ------------------------------------------------- bootstrap on MFMA
// With w_A[r][i], w_B[r][j] the multiplicities of pattern i (j) in resample
// r, Ycount[r][t-1] = sum_i sum_j w_A[r][i] w_B[r][j] [bins_ij >= t]
//                   = sum_j w_B[r][j] U_t[r][j],  U_t = W_A T_t,  T_t = [bins >= t].
// U_t is a product on the matrix cores: w_A in bf16 (integers <= 256 are
// exact), T_t as bf16 0/1 built from the bin bytes per threshold, FP32
// accumulation (partial sums are integers <= kA < 2^24: exact); the sum with
// w_B is taken in integers.  A workgroup owns 32 resamples x 32 columns j;
// wave w owns thresholds 8 w + 1 .. 8 w + 8.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
int g_boot_mfma = 1;         // 0: always the gather kernel (cil_set_option)
void set_boot_gather(int v) { g_boot_mfma = v ? 0 : 1; }

constexpr int BKC = 128;     // i per LDS stage
constexpr int BTPW = 8;      // thresholds per wavefront (M <= 32)

// Multiplicities of both index lists in one launch: elements e < n_boot kA
// count idxA into cA[r][*] (row length ldA), the rest idxB into cB[r][*]
// (row length nB).  flags[0]: an index out of range; flags[1]: a count of
// cA above 256 (not exact in bf16).
__global__ void k_multiplicity(const int *idxA, int kA, long long nA, int ldA, int *cA, const int *idxB, int kB,
                               long long nB, int *cB, int n_boot, int *flags)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long eA = (long long)n_boot * kA;
    if (e >= eA + (long long)n_boot * kB) return;
    const bool isA = e < eA;
    const long long f = isA ? e : e - eA;
    const int k = isA ? kA : kB;
    const long long r = f / k;
    const int v = (isA ? idxA : idxB)[f];
    if (v < 0 || v >= (isA ? nA : nB)) {
        atomicOr(&flags[0], 1);
        return;
    }
    if (isA) {
        if (atomicAdd(&cA[r * ldA + v], 1) >= 256) atomicOr(&flags[1], 1);
    } else {
        atomicAdd(&cB[r * nB + v], 1);
    }
}

// 8 bin bytes -> 8 bf16 values [byte >= t] (bytes and t below 128): the high
// bit of (byte | 0x80) - t marks byte >= t; v_perm moves bytes 0..3 into the
// low byte of 16-bit halves and 0x80 * 0x7f = 0x3f80 is bf16 1.0.
__device__ __forceinline__ bf16x8_t thermometer(uint2 b, unsigned t)
{
    const unsigned tt = t * 0x01010101u;
    const unsigned m0 = ((b.x | 0x80808080u) - tt) & 0x80808080u;
    const unsigned m1 = ((b.y | 0x80808080u) - tt) & 0x80808080u;
    unsigned d[4];
    d[0] = __builtin_amdgcn_perm(0u, m0, 0x0c010c00u) * 0x7fu;
    d[1] = __builtin_amdgcn_perm(0u, m0, 0x0c030c02u) * 0x7fu;
    d[2] = __builtin_amdgcn_perm(0u, m1, 0x0c010c00u) * 0x7fu;
    d[3] = __builtin_amdgcn_perm(0u, m1, 0x0c030c02u) * 0x7fu;
    return __builtin_bit_cast(bf16x8_t, d);
}

__global__ __launch_bounds__(256) void k_boot_mfma(const uint8_t *bins, long long nA, long long nB, int M,
                                                   const int *WA, long long ldA, const int *WB, int n_boot,
                                                   unsigned long long *acc, const int *flags)
{
    if (flags[0] | flags[1]) return;      // an index out of range, or a multiplicity not exact in bf16
    __shared__ __attribute__((aligned(16))) __bf16 sA[32][BKC + 8];     // resample x i
    __shared__ __attribute__((aligned(16))) uint8_t sT[32][BKC + 16];   // column j x i
    __shared__ int sred[4][16][65];                                    // per wavefront: [element][lane]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long long r0 = (long long)blockIdx.y * 32, j0 = (long long)blockIdx.x * 32;
    floatx16_t c[BTPW];
#pragma unroll
    for (int q = 0; q < BTPW; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) c[q][e] = 0.0f;
    for (long long i0 = 0; i0 < nA; i0 += BKC) {
        // every load of the stage is issued before the first store to LDS
        int4 va[2 * (32 * (BKC / 8) / 256)];
        uint8_t vt[BKC * 32 / 256];
#pragma unroll
        for (int q = 0; q < 32 * (BKC / 8) / 256; ++q) {            // W_A rows (zero padded), 8 counts
            const int e = tid + 256 * q, row = e / (BKC / 8), ch = e % (BKC / 8);
            const int4 *src = (const int4 *)(WA + (r0 + row) * ldA + i0 + 8 * ch);
            va[2 * q] = src[0];
            va[2 * q + 1] = src[1];
        }
#pragma unroll
        for (int q = 0; q < BKC * 32 / 256; ++q) {                  // bins rows i, columns j (clamped loads)
            const int e = tid + 256 * q, i = e / 32, j = e % 32;
            const bool in = i0 + i < nA && j0 + j < nB;
            const uint8_t b = bins[min(i0 + i, nA - 1) * nB + min(j0 + j, nB - 1)];
            vt[q] = in ? b : (uint8_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 32 * (BKC / 8) / 256; ++q) {            // counts <= 256: exact in bf16
            const int e = tid + 256 * q, row = e / (BKC / 8), ch = e % (BKC / 8);
            const int4 u = va[2 * q], w = va[2 * q + 1];
            bf16x8_t b;
            b[0] = (__bf16)(float)u.x;
            b[1] = (__bf16)(float)u.y;
            b[2] = (__bf16)(float)u.z;
            b[3] = (__bf16)(float)u.w;
            b[4] = (__bf16)(float)w.x;
            b[5] = (__bf16)(float)w.y;
            b[6] = (__bf16)(float)w.z;
            b[7] = (__bf16)(float)w.w;
            *(bf16x8_t *)&sA[row][8 * ch] = b;
        }
#pragma unroll
        for (int q = 0; q < BKC * 32 / 256; ++q) {                  // -> sT[j][i]
            const int e = tid + 256 * q, i = e / 32, j = e % 32;
            sT[j][i] = vt[q];
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < BKC; kk += 16) {
            const int kofs = kk + 8 * (lane >> 5);
            const bf16x8_t a = *(const bf16x8_t *)&sA[lane & 31][kofs];
            const uint2 braw = *(const uint2 *)&sT[lane & 31][kofs];
#pragma unroll
            for (int q = 0; q < BTPW; ++q) {
                const int t = wv * BTPW + q + 1;
                if (t <= M) c[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, thermometer(braw, t), c[q], 0, 0, 0);
            }
        }
    }
    // C[row][col] = U_t[r0 + row][j0 + col]; element e of lane l: row 8 (e/4) + 4 (l/32) + e%4, col l%32
    const long long j = j0 + (lane & 31);
    int wb[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const long long r = r0 + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
        const int w = WB[min(r, (long long)n_boot - 1) * nB + min(j, nB - 1)];     // clamped: all loads in flight
        wb[e] = (r < n_boot && j < nB) ? w : 0;
    }
    // Row sums over the 32 columns of each half go through this wavefront's
    // slice of LDS: per threshold every lane stores its 16 weighted counts,
    // then lane k < 32 adds the 32 values of (element k / 2, half k % 2) and
    // issues one atomic.  Only this wavefront touches its slice, and a
    // wavefront's LDS accesses are performed in issue order, so a wavefront
    // barrier (no code motion across it) is the only ordering needed.
#pragma unroll
    for (int q = 0; q < BTPW; ++q) {
        const int t = wv * BTPW + q + 1;
        if (t > M) break;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int e = 0; e < 16; ++e) sred[wv][e][lane] = (int)c[q][e] * wb[e];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < 32) {
            const int e = lane >> 1, hf = lane & 1;
            const int *row = &sred[wv][e][32 * hf];
            int v = 0;
#pragma unroll
            for (int k = 0; k < 32; ++k) v += row[k];
            const long long r = r0 + 8 * (e / 4) + 4 * hf + (e % 4);
            if (r < n_boot && v) atomicAdd(&acc[r * M + (t - 1)], (unsigned long long)v);
        }
    }
}

// Device memory of one bootstrap call: the library's grow-only workspaces,
// or (the allocation-free entry point) a fixed region carved in order.
struct BootMem {
    char *base = nullptr;           // null: workspaces
    size_t cap = 0, used = 0;
    // timing marks create HIP events: none on the allocation-free path
    ProfMark mark(const char *name, hipStream_t st) const { return base ? ProfMark{} : prof_begin(name, st); }
    int get(int slot, size_t bytes, void **p)
    {
        if (!base) return ws_get(slot, bytes, p);
        const size_t off = (used + 255) & ~(size_t)255;
        if (off + bytes > cap) return set_error(CIL_EINVAL, "bootstrap scratch of %zu bytes exceeds %zu", off + bytes, cap);
        *p = base + off;
        used = off + bytes;
        return CIL_OK;
    }
};

// One device region per call: the resample counters acc[n_boot M], four
// flag words (gather-path index error, index error, count above 256, pad)
// and, for the matrix-core path, the multiplicities cA[nbP][ldA] and
// cB[n_boot][nB]; cleared by one kernel.
struct BootLayout {
    long long n, nbP, ldA;
    size_t off_flags, off_cA, off_cB, clear, total;
};

static BootLayout boot_layout(long long nA, long long nB, int M, int n_boot, bool mfma)
{
    BootLayout L;
    L.n = (long long)n_boot * M;
    L.nbP = (n_boot + 31) / 32 * 32;
    L.ldA = (nA + BKC - 1) / BKC * BKC;
    L.off_flags = sizeof(unsigned long long) * (size_t)L.n;
    L.off_cA = (L.off_flags + 4 * sizeof(int) + 15) & ~(size_t)15;     // 16-byte rows for the staging loads
    L.off_cB = L.off_cA + (mfma ? sizeof(int) * (size_t)(L.nbP * L.ldA) : 0);
    L.total = L.off_cB + (mfma ? sizeof(int) * (size_t)n_boot * nB : 0);
    L.clear = L.total;
    return L;
}

static bool boot_uses_mfma(int M) { return M <= 4 * BTPW && g_boot_mfma; }

static int bootstrap_run(const uint8_t *bins, long long nA, long long nB, int M, const int *idxA, int kA,
                         const int *idxB, int kB, int n_boot, long long *Ycount, double *Y, hipStream_t st,
                         BootMem &mem, int **defer_flags = nullptr)
{
    const bool work = n_boot > 0 && kA > 0 && kB > 0;
    const bool mfma = work && boot_uses_mfma(M);
    const BootLayout L = boot_layout(nA, nB, M, n_boot, mfma);
    void *p;
    CIL_TRY(mem.get(WS_BOOT_MISC, L.total, &p));
    char *base = (char *)p;
    unsigned long long *acc = (unsigned long long *)base;
    int *flags = (int *)(base + L.off_flags);
    CIL_TRY(fill_zero(base, L.clear, st));
    if (mfma) {
        // the matrix-core path runs unless an index is out of range
        // (flags[1]) or a multiplicity exceeds 256 (flags[2], possible only
        // for kA > 256): the kernel checks both itself, and a gather launch
        // follows that runs only if it declined
        int *cA = (int *)(base + L.off_cA), *cB = (int *)(base + L.off_cB);
        const long long tot = (long long)n_boot * (kA + kB);
        hipLaunchKernelGGL(k_multiplicity, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, idxA, kA, nA,
                           (int)L.ldA, cA, idxB, kB, nB, cB, n_boot, flags + 1);
        CIL_TRY(check_launch("k_multiplicity"));
        dim3 grid((unsigned)((nB + 31) / 32), (unsigned)(L.nbP / 32));
        const ProfMark pm = mem.mark("k_bootstrap", st);
        hipLaunchKernelGGL(k_boot_mfma, grid, dim3(256), 0, st, bins, nA, nB, M, cA, L.ldA, cB, n_boot, acc,
                           flags + 1);
        prof_end(pm, st);
        CIL_TRY(check_launch("k_boot_mfma"));
    }
    if (work && (!mfma || kA > 256)) {
        // gather path (after the matrix-core kernel: only if that declined);
        // the kA rows of a resample are split over enough blocks to fill the chip
        const int *only_if = mfma ? flags + 1 : nullptr;
        int slices = (int)std::max<long long>(1, std::min<long long>(kA, (2048 + n_boot - 1) / n_boot));
        const int rpb = (kA + slices - 1) / slices;
        slices = (kA + rpb - 1) / rpb;
        const size_t shmem = sizeof(int) * (size_t)kB + sizeof(unsigned int) * 256;
        dim3 grid(slices, n_boot);
        if (shmem > 160 * 1024) return set_error(CIL_EUNSUPPORTED, "kB too large for the bootstrap kernel");
        const ProfMark pm = mem.mark("k_bootstrap", st);
        if (M <= 16)
            hipLaunchKernelGGL(k_bootstrap<16>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc,
                               flags, only_if);
        else if (M <= 32)
            hipLaunchKernelGGL(k_bootstrap<32>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc,
                               flags, only_if);
        else if (M <= 64)
            hipLaunchKernelGGL(k_bootstrap<64>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc,
                               flags, only_if);
        else
            hipLaunchKernelGGL(k_bootstrap_hist, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb,
                               acc, flags, only_if);
        prof_end(pm, st);
        CIL_TRY(check_launch("k_bootstrap"));
    }
    const double denom = (double)kA * (double)kB;
    if (L.n > 0) {
        hipLaunchKernelGGL(k_boot_finish, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, acc, L.n, denom, Ycount,
                           Y);
        CIL_TRY(check_launch("k_boot_finish"));
    }
    if (defer_flags) {                 // the caller reads the two index flags later
        *defer_flags = flags;
        return CIL_OK;
    }
    // pinned host words keep the copy asynchronous; the allocation-free path
    // reads into the stack instead (pinned memory would be allocated)
    int hloc[2];
    int *hbad = hloc;
    if (!mem.base) CIL_TRY(host_stage(HS_BOOT, 2 * sizeof(int), (void **)&hbad));
    hbad[0] = hbad[1] = 0;
    CIL_HIP(hipMemcpyAsync(hbad, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    CIL_TRY(stream_wait(st));
    if (hbad[0] || hbad[1]) return set_error(CIL_EINVAL, "bootstrap index out of range");
    return CIL_OK;
}

int bootstrap_impl(const uint8_t *bins, long long nA, long long nB, int M, const int *idxA, int kA,
                   const int *idxB, int kB, int n_boot, long long *Ycount, double *Y, hipStream_t st)
{
    BootMem mem;
    return bootstrap_run(bins, nA, nB, M, idxA, kA, idxB, kB, n_boot, Ycount, Y, st, mem);
}

// The bootstrap without its index-flag read-back; *flags (device int[2],
// nonzero: an index out of range) is left for the caller to read.
int bootstrap_deferred(const uint8_t *bins, long long nA, long long nB, int M, const int *idxA, int kA,
                       const int *idxB, int kB, int n_boot, double *Y, hipStream_t st, int **flags)
{
    BootMem mem;
    return bootstrap_run(bins, nA, nB, M, idxA, kA, idxB, kB, n_boot, nullptr, Y, st, mem, flags);
}

// The observed correlation integral vector from a bin histogram (hist[m]:
// pairs in bin m, m = 0..M): y[m - 1] = #{pairs with bin >= m} / denom, the
// counts accumulated from the top bin down as integers, then one division.
__global__ void k_observed(const unsigned long long *hist, int M, double denom, double *y)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long run = 0;
    for (int m = M; m >= 1; --m) {
        run += hist[m];
        y[m - 1] = (double)run / denom;
    }
}

int observed_from_hist(const unsigned long long *hist, int M, double denom, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_observed, dim3(1), dim3(64), 0, st, hist, M, denom, y);
    return check_launch("k_observed");
}

// ------------------------------------- bootstrap without allocation
// For callers that cannot allocate device memory: the bootstrap's counters,
// multiplicities and flags live in this fixed per-device array instead of
// the library's workspaces.  Host code never passes the array's name to a
// kernel: its device address comes from hipGetSymbolAddress, once per device.
constexpr size_t BOOT_NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;   // 16 MiB per device
static __device__ __align__(256) char scratch[BOOT_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, char *> g_scratch_ptr;

static int scratch_address(char **out)
{
    int dev;
    CIL_TRY(current_device(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return set_error(CIL_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        it = g_scratch_ptr.emplace(dev, (char *)ptr).first;
    }
    *out = it->second;
    return CIL_OK;
}

size_t bootstrap_noalloc_bytes(long long nA, long long nB, int M, int n_boot)
{
    return boot_layout(nA, nB, M, n_boot, boot_uses_mfma(M)).total;
}

int bootstrap_noalloc_impl(const uint8_t *bins, long long nA, long long nB, int M, const int *idxA, int kA,
                           const int *idxB, int kB, int n_boot, long long *Ycount, double *Y, hipStream_t st)
{
    const size_t need = bootstrap_noalloc_bytes(nA, nB, M, n_boot);
    if (need > BOOT_NOALLOC_SCRATCH_BYTES)
        return set_error(CIL_EINVAL, "the allocation-free bootstrap needs %zu bytes of scratch, its maximum is %zu",
                         need, (size_t)BOOT_NOALLOC_SCRATCH_BYTES);
    BootMem mem;
    CIL_TRY(scratch_address(&mem.base));
    mem.cap = BOOT_NOALLOC_SCRATCH_BYTES;
    return bootstrap_run(bins, nA, nB, M, idxA, kA, idxB, kB, n_boot, Ycount, Y, st, mem);
}

// ---------------------------------------------------------- likelihood
// One workgroup per problem.  mu and Sigma two-pass (1/(n-1)); bins with a
// sample variance of exactly 0 are dropped; Cholesky-Banachiewicz on the
// kept bins in LDS; z = L^-1 (y - mu); f = |z|^2; loglik = -f/2 - sum log L_ii
// - (m_eff/2) log 2 pi.  FP64 throughout.  The resample vectors are staged in
// LDS by coalesced loads, as many rows at a time as fit (all of them for
// M <= 15 and n <= 200); every sum still runs over the rows in order, so the
// mean, the covariance and the dropped-bin decision are those of a plain
// sequential two-pass evaluation.
constexpr int LMAX = 64;
constexpr int YSTAGE = 3072;                 // doubles of resample rows staged per chunk

__global__ __launch_bounds__(256) void k_loglik(const double *Y, int n, int M, const double *yobs,
                                                double *f, double *loglik, int *meff, int *status)
{
    constexpr int NE = (LMAX * (LMAX + 1) / 2 + 255) / 256;  // covariance entries per thread
    __shared__ double mu[LMAX];
    __shared__ double S[LMAX][LMAX + 1];
    __shared__ double Ys[YSTAGE];
    __shared__ int keep[LMAX];
    __shared__ int nk;
    __shared__ double z[LMAX];
    __shared__ double lgd[LMAX];
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    const double *Yp = Y + (size_t)p * n * M;
    const int RC = YSTAGE / M;                               // rows per chunk (>= 48)
    const bool resident = n <= RC;                           // every row fits at once

    // pass 1: mean, each bin summed over the rows in order
    double s = 0.0;
    for (int r0 = 0; r0 < n; r0 += RC) {
        const int cnt = min(RC, n - r0) * M;
        __syncthreads();
        for (int q0 = lane; q0 < cnt; q0 += 256 * 8) {     // eight unconditional loads in flight per thread
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = Yp[(size_t)r0 * M + min(q0 + 256 * u, cnt - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q0 + 256 * u < cnt) Ys[q0 + 256 * u] = v[u];
        }
        __syncthreads();
        if (lane < M) {
            int q = lane;
            for (; q + 7 * M < cnt; q += 8 * M) {       // eight loads in flight, added in row order
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = Ys[q + u * M];
#pragma unroll
                for (int u = 0; u < 8; ++u) s += v[u];
            }
            for (; q < cnt; q += M) s += Ys[q];
        }
    }
    if (lane < M) mu[lane] = s / n;
    __syncthreads();
    // covariance entries (i, j), i >= j, spread over the threads; each entry
    // sums the products of the centred rows in order
    const int ne = M * (M + 1) / 2;
    double acc[NE];
    int ei[NE], ej[NE];
#pragma unroll
    for (int t = 0; t < NE; ++t) {
        acc[t] = 0.0;
        const int e = lane + 256 * t;
        int i = 0;
        if (e < ne) {
            i = (int)((sqrt(8.0 * e + 1.0) - 1.0) / 2.0);
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            while (i * (i + 1) / 2 > e) --i;
        }
        ei[t] = i;
        ej[t] = e < ne ? e - i * (i + 1) / 2 : 0;
    }
    for (int r0 = 0; r0 < n; r0 += RC) {
        const int rows = min(RC, n - r0);
        if (resident) {                                      // centre the staged rows in place
            for (int q = lane; q < rows * M; q += 256) Ys[q] -= mu[q % M];
        } else {
            __syncthreads();
            for (int q0 = lane; q0 < rows * M; q0 += 256 * 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = Yp[(size_t)r0 * M + min(q0 + 256 * u, rows * M - 1)];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (q0 + 256 * u < rows * M) Ys[q0 + 256 * u] = v[u] - mu[(q0 + 256 * u) % M];
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NE; ++t)
            if (lane + 256 * t < ne) {
                const double *a = Ys + ei[t], *b = Ys + ej[t];
                int r = 0;
                for (; r + 8 <= rows; r += 8) {             // eight row pairs in flight, added in row order
                    double x[8], y[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        x[u] = a[(r + u) * M];
                        y[u] = b[(r + u) * M];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[t] += x[u] * y[u];
                }
                for (; r < rows; ++r) acc[t] += a[r * M] * b[r * M];
            }
    }
#pragma unroll
    for (int t = 0; t < NE; ++t)
        if (lane + 256 * t < ne) {
            const double sv = acc[t] / (n - 1);
            S[ei[t]][ej[t]] = sv;
            S[ej[t]][ei[t]] = sv;
        }
    __syncthreads();
    // From here one wavefront works alone: its LDS accesses are performed in
    // issue order, so a wavefront barrier (no code motion across it) orders
    // them; the other wavefronts leave.
    if (lane >= 64) return;
    auto wsync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    if (lane == 0) {
        int c = 0;
        for (int m = 0; m < M; ++m)
            if (S[m][m] != 0.0) keep[c++] = m;
        nk = c;
    }
    wsync();
    const int K = nk;
    if (K <= 16) {
        // Up to 16 kept bins: lane i holds row i of Sigma in registers and
        // reads other lanes' entries with readlane, so no step waits on the
        // LDS.  Right-looking Cholesky and solve: every entry subtracts its
        // terms in index order, the operations of the left-looking form.
        constexpr int R = 16;
        auto bcast = [](double x, int src) {               // src is a compile-time lane after unrolling
            const long long v = __double_as_longlong(x);
            const int lo = __builtin_amdgcn_readlane((int)v, src);
            const int hi = __builtin_amdgcn_readlane((int)(v >> 32), src);
            return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
        };
        const int kl = lane < K ? keep[lane] : 0;
        double r[R];
#pragma unroll
        for (int j = 0; j < R; ++j) r[j] = (lane < K && j < K) ? S[kl][keep[j < K ? j : 0]] : 0.0;
        const double dg_own = lane < K ? S[kl][kl] : 0.0;
        double diag_own = 0.0;
        int ok = 1;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (j < K) {
                const double sv = bcast(r[j], j), dgj = bcast(dg_own, j);
                const double d = (sv > K * 0x1p-52 * dgj) ? sqrt(sv) : NAN;
                if (!(d > 0.0)) ok = 0;
                if (lane == j) {
                    r[j] = d;
                    diag_own = d;
                }
                if (lane > j && lane < K) r[j] = r[j] / d;
#pragma unroll
                for (int c = j + 1; c < R; ++c) {
                    if (c < K) {
                        const double lcj = bcast(r[j], c);
                        if (lane >= c && lane < K) r[c] -= r[j] * lcj;
                    }
                }
            }
        }
        const double lg_own = (ok && lane < K) ? log(diag_own) : 0.0;
        double rhs = lane < K ? yobs[(size_t)p * M + kl] - mu[kl] : 0.0;
        double acc = 0.0, ld = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k < K) {
                const double zk = bcast(rhs, k) / bcast(diag_own, k);
                if (lane > k && lane < K) rhs -= r[k] * zk;
                acc += zk * zk;
                ld += bcast(lg_own, k);
            }
        }
        if (lane == 0) {
            f[p] = ok ? acc : NAN;
            loglik[p] = ok ? -0.5 * acc - ld - 0.5 * K * log(2.0 * M_PI) : NAN;
            meff[p] = K;
            status[p] = ok ? CIL_OK : CIL_ENOTSPD;
        }
        return;
    }
    // compact the kept rows/columns into the leading K x K block (in place:
    // keep[] is increasing so keep[a] >= a); lane c moves column c
    for (int a = 0; a < K; ++a) {
        double v = 0.0;
        if (lane < K) v = S[keep[a]][keep[lane]];
        wsync();
        if (lane < K) S[a][lane] = v;
        wsync();
    }
    // Cholesky, lower triangle in S; a pivot not above K 2^-52 Sigma_jj means
    // Sigma is singular to working precision.  The dot products subtract
    // their terms in index order; the loads run four ahead.
    auto dot_sub = [](double s, const double *x, const double *y, int len) {
        int k = 0;
        for (; k + 4 <= len; k += 4) {
            const double x0 = x[k], x1 = x[k + 1], x2 = x[k + 2], x3 = x[k + 3];
            const double y0 = y[k], y1 = y[k + 1], y2 = y[k + 2], y3 = y[k + 3];
            s -= x0 * y0;
            s -= x1 * y1;
            s -= x2 * y2;
            s -= x3 * y3;
        }
        for (; k < len; ++k) s -= x[k] * y[k];
        return s;
    };
    int ok = 1;
    for (int j = 0; j < K; ++j) {
        if (lane == 0) {
            const double diag = S[j][j];
            const double sv = dot_sub(diag, S[j], S[j], j);
            S[j][j] = (sv > K * 0x1p-52 * diag) ? sqrt(sv) : NAN;
        }
        wsync();
        const double d = S[j][j];
        if (!(d > 0.0)) ok = 0;
        if (lane > j && lane < K) S[lane][j] = dot_sub(S[lane][j], S[lane], S[j], j) / d;
        wsync();
    }
    if (lane < K) lgd[lane] = ok ? log(S[lane][lane]) : 0.0;   // the logs in parallel, summed in order below
    wsync();
    if (lane == 0) {
        double ff = NAN, ll = NAN;
        if (ok) {
            double acc = 0.0, ld = 0.0;
            for (int i = 0; i < K; ++i) {
                const double sv = dot_sub(yobs[(size_t)p * M + keep[i]] - mu[keep[i]], S[i], z, i);
                z[i] = sv / S[i][i];
                acc += z[i] * z[i];
                ld += lgd[i];
            }
            ff = acc;
            ll = -0.5 * acc - ld - 0.5 * K * log(2.0 * M_PI);
        }
        f[p] = ff;
        loglik[p] = ll;
        meff[p] = K;
        status[p] = ok ? CIL_OK : CIL_ENOTSPD;
    }
}

int loglik_impl(const double *Y, int P, int n, int M, const double *yobs, double *f, double *ll, int *meff,
                int *status, hipStream_t st)
{
    if (P <= 0) return CIL_OK;
    const ProfMark pm = prof_begin("k_loglik", st);
    hipLaunchKernelGGL(k_loglik, dim3(P), dim3(256), 0, st, Y, n, M, yobs, f, ll, meff, status);
    prof_end(pm, st);
    return check_launch("k_loglik");
}

}  // namespace cil
