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

__global__ void k_multiplicity(const int *idx, int k, int n_boot, long long n, int ld, int *cnt, int *bad)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n_boot * k) return;
    const long long r = e / k;
    const int v = idx[e];
    if (v < 0 || v >= n) {
        atomicOr(bad, 1);
        return;
    }
    atomicAdd(&cnt[r * ld + v], 1);
}

__global__ void k_mult_to_bf16(const int *cnt, long long total, __bf16 *w, int *over)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int v = cnt[e];
    if (v > 256) atomicOr(over, 1);
    w[e] = (__bf16)(float)v;
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
                                                   const __bf16 *WA, long long ldA, const int *WB, int n_boot,
                                                   unsigned long long *acc, const int *flags)
{
    if (flags[0] | flags[1]) return;      // an index out of range, or a multiplicity not exact in bf16
    __shared__ __attribute__((aligned(16))) __bf16 sA[32][BKC + 8];     // resample x i
    __shared__ __attribute__((aligned(16))) uint8_t sT[32][BKC + 16];   // column j x i
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long long r0 = (long long)blockIdx.y * 32, j0 = (long long)blockIdx.x * 32;
    floatx16_t c[BTPW];
#pragma unroll
    for (int q = 0; q < BTPW; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) c[q][e] = 0.0f;
    for (long long i0 = 0; i0 < nA; i0 += BKC) {
        // every load of the stage is issued before the first store to LDS
        bf16x8_t va[32 * (BKC / 8) / 256];
        uint8_t vt[BKC * 32 / 256];
#pragma unroll
        for (int q = 0; q < 32 * (BKC / 8) / 256; ++q) {            // W_A rows (zero padded)
            const int e = tid + 256 * q, row = e / (BKC / 8), ch = e % (BKC / 8);
            va[q] = *(const bf16x8_t *)(WA + (r0 + row) * ldA + i0 + 8 * ch);
        }
#pragma unroll
        for (int q = 0; q < BKC * 32 / 256; ++q) {                  // bins rows i, columns j
            const int e = tid + 256 * q, i = e / 32, j = e % 32;
            vt[q] = (i0 + i < nA && j0 + j < nB) ? bins[(i0 + i) * nB + j0 + j] : (uint8_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 32 * (BKC / 8) / 256; ++q) {
            const int e = tid + 256 * q, row = e / (BKC / 8), ch = e % (BKC / 8);
            *(bf16x8_t *)&sA[row][8 * ch] = va[q];
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
        wb[e] = (r < n_boot && j < nB) ? WB[r * nB + j] : 0;
    }
#pragma unroll
    for (int q = 0; q < BTPW; ++q) {
        const int t = wv * BTPW + q + 1;
        if (t > M) break;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            int v = (int)c[q][e] * wb[e];
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);   // over the 32 columns of this half
            const long long r = r0 + 8 * (e / 4) + 4 * (lane >> 5) + (e % 4);
            if ((lane & 31) == 0 && r < n_boot && v) atomicAdd(&acc[r * M + (t - 1)], (unsigned long long)v);
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

size_t boot_mult_bytes(long long nA, long long nB, int n_boot)
{
    const long long nbP = (n_boot + 31) / 32 * 32, ldA = (nA + BKC - 1) / BKC * BKC;
    return sizeof(int) * (size_t)(nbP * ldA) + sizeof(int) * (size_t)n_boot * nB + sizeof(__bf16) * (size_t)(nbP * ldA) +
           64;
}

// MFMA path.  It runs unless an index is out of range (flags[0]) or a
// multiplicity exceeds 256 (flags[1], possible only for kA > 256): both are
// known on the device only, so the kernel checks them itself; *flags_out
// points at them for a gather launch that runs only when the MFMA kernel
// declined (*may_decline).
int bootstrap_mfma(const uint8_t *bins, long long nA, long long nB, int M, const int *idxA, int kA, const int *idxB,
                   int kB, int n_boot, unsigned long long *acc, hipStream_t st, const int **flags_out,
                   bool *may_decline, BootMem &mem)
{
    const long long nbP = (n_boot + 31) / 32 * 32, ldA = (nA + BKC - 1) / BKC * BKC;
    const size_t szA = sizeof(int) * (size_t)(nbP * ldA), szB = sizeof(int) * (size_t)n_boot * nB;
    const size_t szW = sizeof(__bf16) * (size_t)(nbP * ldA);
    void *p;
    CIL_TRY(mem.get(WS_BOOT_MULT, boot_mult_bytes(nA, nB, n_boot), &p));
    int *cA = (int *)p;
    int *cB = cA + nbP * ldA;
    __bf16 *wA = (__bf16 *)(cB + (size_t)n_boot * nB);
    int *flags = (int *)((char *)wA + szW);          // bad, over
    CIL_TRY(fill_zero(cA, szA + szB, st));
    CIL_TRY(fill_zero(flags, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_multiplicity, dim3((unsigned)(((long long)n_boot * kA + 255) / 256)), dim3(256), 0, st, idxA,
                       kA, n_boot, nA, (int)ldA, cA, flags);
    hipLaunchKernelGGL(k_multiplicity, dim3((unsigned)(((long long)n_boot * kB + 255) / 256)), dim3(256), 0, st, idxB,
                       kB, n_boot, nB, (int)nB, cB, flags);
    hipLaunchKernelGGL(k_mult_to_bf16, dim3((unsigned)((nbP * ldA + 255) / 256)), dim3(256), 0, st, cA, nbP * ldA, wA,
                       flags + 1);
    CIL_TRY(check_launch("k_multiplicity"));
    dim3 grid((unsigned)((nB + 31) / 32), (unsigned)(nbP / 32));
    const ProfMark pm = mem.mark("k_bootstrap", st);
    hipLaunchKernelGGL(k_boot_mfma, grid, dim3(256), 0, st, bins, nA, nB, M, wA, ldA, cB, n_boot, acc, flags);
    prof_end(pm, st);
    CIL_TRY(check_launch("k_boot_mfma"));
    *flags_out = flags;
    *may_decline = kA > 256;
    return CIL_OK;
}

static bool boot_uses_mfma(int M) { return M <= 4 * BTPW && g_boot_mfma; }

static int bootstrap_run(const uint8_t *bins, long long nA, long long nB, int M, const int *idxA, int kA,
                         const int *idxB, int kB, int n_boot, long long *Ycount, double *Y, hipStream_t st,
                         BootMem &mem)
{
    void *p;
    const long long n = (long long)n_boot * M;
    CIL_TRY(mem.get(WS_BOOT_MISC, sizeof(unsigned long long) * (size_t)(n + 1), &p));
    unsigned long long *acc = (unsigned long long *)p;
    int *bad = (int *)(acc + n);
    CIL_TRY(fill_zero(acc, sizeof(unsigned long long) * (size_t)(n + 1), st));
    const bool work = n_boot > 0 && kA > 0 && kB > 0;
    bool mfma = false, may_decline = false;
    const int *mflags = nullptr;
    if (work && boot_uses_mfma(M)) {
        CIL_TRY(bootstrap_mfma(bins, nA, nB, M, idxA, kA, idxB, kB, n_boot, acc, st, &mflags, &may_decline, mem));
        mfma = true;
    }
    if (work && (!mfma || may_decline)) {
        // gather path (after the MFMA kernel: only if that declined); the kA
        // rows of a resample are split over enough blocks to fill the chip
        const int *only_if = mfma ? mflags : nullptr;
        int slices = (int)std::max<long long>(1, std::min<long long>(kA, (2048 + n_boot - 1) / n_boot));
        const int rpb = (kA + slices - 1) / slices;
        slices = (kA + rpb - 1) / rpb;
        const size_t shmem = sizeof(int) * (size_t)kB + sizeof(unsigned int) * 256;
        dim3 grid(slices, n_boot);
        if (shmem > 160 * 1024) return set_error(CIL_EUNSUPPORTED, "kB too large for the bootstrap kernel");
        const ProfMark pm = mem.mark("k_bootstrap", st);
        if (M <= 16)
            hipLaunchKernelGGL(k_bootstrap<16>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc,
                               bad, only_if);
        else if (M <= 32)
            hipLaunchKernelGGL(k_bootstrap<32>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc,
                               bad, only_if);
        else if (M <= 64)
            hipLaunchKernelGGL(k_bootstrap<64>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc,
                               bad, only_if);
        else
            hipLaunchKernelGGL(k_bootstrap_hist, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb,
                               acc, bad, only_if);
        prof_end(pm, st);
        CIL_TRY(check_launch("k_bootstrap"));
    }
    const double denom = (double)kA * (double)kB;
    if (n > 0) {
        hipLaunchKernelGGL(k_boot_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, acc, n, denom, Ycount, Y);
        CIL_TRY(check_launch("k_boot_finish"));
    }
    int hbad[2] = {0, 0};
    CIL_HIP(hipMemcpyAsync(&hbad[0], bad, sizeof(int), hipMemcpyDeviceToHost, st));
    if (mflags) CIL_HIP(hipMemcpyAsync(&hbad[1], mflags, sizeof(int), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    if (hbad[0] || hbad[1]) return set_error(CIL_EINVAL, "bootstrap index out of range");
    return CIL_OK;
}

int bootstrap_impl(const uint8_t *bins, long long nA, long long nB, int M, const int *idxA, int kA,
                   const int *idxB, int kB, int n_boot, long long *Ycount, double *Y, hipStream_t st)
{
    BootMem mem;
    return bootstrap_run(bins, nA, nB, M, idxA, kA, idxB, kB, n_boot, Ycount, Y, st, mem);
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
    const size_t acc = sizeof(unsigned long long) * (size_t)((long long)n_boot * M + 1);
    size_t total = acc;
    if (boot_uses_mfma(M)) total = ((total + 255) & ~(size_t)255) + boot_mult_bytes(nA, nB, n_boot);
    return total;
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
        for (int q = lane; q < cnt; q += 256) Ys[q] = Yp[(size_t)r0 * M + q];
        __syncthreads();
        if (lane < M)
            for (int q = lane; q < cnt; q += M) s += Ys[q];
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
            for (int q = lane; q < rows * M; q += 256) Ys[q] = Yp[(size_t)r0 * M + q] - mu[q % M];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NE; ++t)
            if (lane + 256 * t < ne) {
                const double *a = Ys + ei[t], *b = Ys + ej[t];
                for (int r = 0; r < rows; ++r) acc[t] += a[r * M] * b[r * M];
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
    if (lane == 0) {
        int c = 0;
        for (int m = 0; m < M; ++m)
            if (S[m][m] != 0.0) keep[c++] = m;
        nk = c;
    }
    __syncthreads();
    const int K = nk;
    // compact the kept rows/columns into the leading K x K block (in place:
    // keep[] is increasing so keep[a] >= a)
    for (int a = 0; a < K; ++a) {
        double v = 0.0;
        if (lane < K) v = S[keep[a]][keep[lane]];
        __syncthreads();
        if (lane < K) S[a][lane] = v;
        __syncthreads();
    }
    // Cholesky, lower triangle in S; a pivot not above K 2^-52 Sigma_jj means
    // Sigma is singular to working precision
    int ok = 1;
    for (int j = 0; j < K; ++j) {
        if (lane == 0) {
            const double diag = S[j][j];
            double s = diag;
            for (int k = 0; k < j; ++k) s -= S[j][k] * S[j][k];
            S[j][j] = (s > K * 0x1p-52 * diag) ? sqrt(s) : NAN;
        }
        __syncthreads();
        const double d = S[j][j];
        if (!(d > 0.0)) ok = 0;
        if (lane > j && lane < K) {
            double s = S[lane][j];
            for (int k = 0; k < j; ++k) s -= S[lane][k] * S[j][k];
            S[lane][j] = s / d;
        }
        __syncthreads();
    }
    if (lane == 0) {
        double ff = NAN, ll = NAN;
        if (ok) {
            double acc = 0.0, ld = 0.0;
            for (int i = 0; i < K; ++i) {
                double s = yobs[(size_t)p * M + keep[i]] - mu[keep[i]];
                for (int k = 0; k < i; ++k) s -= S[i][k] * z[k];
                z[i] = s / S[i][i];
                acc += z[i] * z[i];
                ld += log(S[i][i]);
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
