// Bootstrap correlation integral vectors (Alg. 2bst / Alg. 3bst step 2) and
// the Gaussian synthetic likelihood (eqs. cil:CF, cil:CF_synth) on gfx950.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>

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
                                                   int *bad)
{
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
                                                        int rows_per_block, unsigned long long *Ycnt, int *bad)
{
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

int bootstrap_impl(const uint8_t *bins, long long nA, long long nB, int M, const int *idxA, int kA,
                   const int *idxB, int kB, int n_boot, long long *Ycount, double *Y, hipStream_t st)
{
    void *p;
    const long long n = (long long)n_boot * M;
    CIL_TRY(ws_get(WS_BOOT_MISC, sizeof(unsigned long long) * (size_t)(n + 1), &p));
    unsigned long long *acc = (unsigned long long *)p;
    int *bad = (int *)(acc + n);
    CIL_TRY(fill_zero(acc, sizeof(unsigned long long) * (size_t)(n + 1), st));
    if (n_boot > 0 && kA > 0 && kB > 0) {
        // split the kA rows of a resample over enough blocks to fill the chip
        int slices = (int)std::max<long long>(1, std::min<long long>(kA, (2048 + n_boot - 1) / n_boot));
        const int rpb = (kA + slices - 1) / slices;
        slices = (kA + rpb - 1) / rpb;
        const size_t shmem = sizeof(int) * (size_t)kB + sizeof(unsigned int) * 256;
        dim3 grid(slices, n_boot);
        if (shmem > 160 * 1024) return set_error(CIL_EUNSUPPORTED, "kB too large for the bootstrap kernel");
        const ProfMark pm = prof_begin("k_bootstrap", st);
        if (M <= 16)
            hipLaunchKernelGGL(k_bootstrap<16>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc, bad);
        else if (M <= 32)
            hipLaunchKernelGGL(k_bootstrap<32>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc, bad);
        else if (M <= 64)
            hipLaunchKernelGGL(k_bootstrap<64>, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc, bad);
        else
            hipLaunchKernelGGL(k_bootstrap_hist, grid, dim3(256), shmem, st, bins, nA, nB, M, idxA, kA, idxB, kB, rpb, acc, bad);
        prof_end(pm, st);
        CIL_TRY(check_launch("k_bootstrap"));
    }
    const double denom = (double)kA * (double)kB;
    if (n > 0) {
        hipLaunchKernelGGL(k_boot_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, acc, n, denom, Ycount, Y);
        CIL_TRY(check_launch("k_boot_finish"));
    }
    int hbad = 0;
    CIL_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipStreamSynchronize(st));
    if (hbad) return set_error(CIL_EINVAL, "bootstrap index out of range");
    return CIL_OK;
}

// ---------------------------------------------------------- likelihood
// One wavefront per problem.  mu and Sigma two-pass (1/(n-1)); bins with a
// sample variance of exactly 0 are dropped; Cholesky-Banachiewicz on the
// kept bins in LDS; z = L^-1 (y - mu); f = |z|^2; loglik = -f/2 - sum log L_ii
// - (m_eff/2) log 2 pi.  FP64 throughout.
constexpr int LMAX = 64;

__global__ __launch_bounds__(256) void k_loglik(const double *Y, int n, int M, const double *yobs,
                                                double *f, double *loglik, int *meff, int *status)
{
    constexpr int RC = 32;                                   // rows staged per chunk
    constexpr int NE = (LMAX * (LMAX + 1) / 2 + 255) / 256;  // covariance entries per thread
    __shared__ double mu[LMAX];
    __shared__ double S[LMAX][LMAX + 1];
    __shared__ double Yc[RC][LMAX];
    __shared__ int keep[LMAX];
    __shared__ int nk;
    __shared__ double z[LMAX];
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    const double *Yp = Y + (size_t)p * n * M;

    if (lane < M) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += Yp[(size_t)r * M + lane];
        mu[lane] = s / n;
    }
    __syncthreads();
    // covariance entries (i, j), i >= j, spread over the threads; the centred
    // rows are staged in LDS a chunk at a time, each entry sums over r in order
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
        for (int q = lane; q < rows * M; q += 256) {
            const int r = q / M, m = q % M;
            Yc[r][m] = Yp[(size_t)(r0 + r) * M + m] - mu[m];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NE; ++t)
            if (lane + 256 * t < ne)
                for (int r = 0; r < rows; ++r) acc[t] += Yc[r][ei[t]] * Yc[r][ej[t]];
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < NE; ++t)
        if (lane + 256 * t < ne) {
            const double s = acc[t] / (n - 1);
            S[ei[t]][ej[t]] = s;
            S[ej[t]][ei[t]] = s;
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
