// Length-N DCT-II and its inverse on one line held in a thread's registers.
//
// The implicit diffusion solve of the IMEX step is diagonal in the cosine
// basis cos(pi k (j + 1/2) / N) of the ghost-copy Neumann Laplacian
// (App. B.1.1), so each step transforms every row and column of the grid.
// Here one thread owns one full line (N = 32, 64 or 128 values) and
// transforms it with Makhoul's reduction of the DCT-II to a length-N real DFT
// (even/odd reordering, then a phase rotation by exp(-i pi k / 2N)), the real
// DFT being one radix-2 complex FFT of length N/2 plus a split step.  Every
// loop is unrolled at compile time, so the indices are constants, the arrays
// stay in VGPRs and all twiddles are instruction literals.
//
// Scaling (folded by the caller into the spectral divisor):
//   forward(x) = 2 * DCT2(x),   DCT2(x)_k = sum_j x_j cos(pi k (2j+1) / 2N)
//   inverse(X) = N * DCT2^{-1}(X)
#pragma once

#include "cil_internal.hpp"

namespace cil {

template <typename T, int N>
struct DctLine {
    static constexpr int M = N / 2;           // complex FFT length
    static constexpr int LOGM = ilog2(M);
    static_assert((1 << LOGM) == M && N >= 8, "N must be a power of two >= 8");

    // Even/odd reordering v_j = x_{2j} (j < M), v_{N-1-j} = x_{2j+1}:
    // the input element that lands at position j of v.
    static constexpr int vsrc(int j) { return j < M ? 2 * j : 2 * (N - 1 - j) + 1; }

    // In-place radix-2 decimation-in-time FFT of length M; input in
    // bit-reversed order, output in natural order.  SIGN = -1 forward,
    // +1 backward (no 1/M).
    template <int SIGN>
    __device__ __forceinline__ static void fft(T (&re)[M], T (&im)[M])
    {
        static_for<1, LOGM + 1>([&](auto S) {
            constexpr int m = 1 << S;
            constexpr int h = m / 2;
            static_for<0, M / m>([&](auto B) {
                constexpr int k0 = B * m;
                static_for<0, h>([&](auto J) {
                    constexpr int j = J;
                    constexpr int a = k0 + j, b = a + h;
                    T tr, ti;
                    if constexpr (j == 0) {
                        tr = re[b];
                        ti = im[b];
                    } else if constexpr (4 * j == m) {     // W = SIGN * i
                        tr = (SIGN > 0) ? -im[b] : im[b];
                        ti = (SIGN > 0) ? re[b] : -re[b];
                    } else {
                        constexpr T wr = (T)ce_cospi(2 * j, m);
                        constexpr T wi = (T)(SIGN * ce_sinpi(2 * j, m));
                        tr = wr * re[b] - wi * im[b];
                        ti = wr * im[b] + wi * re[b];
                    }
                    re[b] = re[a] - tr;
                    im[b] = im[a] - ti;
                    re[a] = re[a] + tr;
                    im[a] = im[a] + ti;
                });
            });
        });
    }

    // X = 2 * DCT2(x).
    __device__ __forceinline__ static void forward(const T (&x)[N], T (&X)[N])
    {
        T zr[M], zi[M];
        static_for<0, M>([&](auto Mi) {
            constexpr int m = Mi;
            constexpr int p = bitrev(m, LOGM);
            zr[p] = x[vsrc(2 * m)];
            zi[p] = x[vsrc(2 * m + 1)];
        });
        fft<-1>(zr, zi);
        // V_k = E_k + e^{-2 pi i k/N} O_k with 2E_k = Z_k + conj(Z_{M-k}),
        // 2O_k = (Z_k - conj(Z_{M-k}))/i; then X_k = Re(e^{-i pi k/2N} V_k),
        // X_{N-k} = -Im(e^{-i pi k/2N} V_k).  (Factors 1/2 dropped: X doubled.)
        static_for<0, M + 1>([&](auto Ki) {
            constexpr int k = Ki;
            constexpr int k1 = k % M, k2 = (M - k) % M;
            const T a = zr[k1], b = zi[k1], c = zr[k2], d = -zi[k2];
            const T Er = a + c, Ei = b + d;
            const T Or = b - d, Oi = c - a;
            constexpr T wr = (T)ce_cospi(2 * k, N);
            constexpr T wi = (T)(-ce_sinpi(2 * k, N));
            const T Vr = Er + (wr * Or - wi * Oi);
            const T Vi = Ei + (wr * Oi + wi * Or);
            constexpr T cph = (T)ce_cospi(k, 2 * N);
            constexpr T sph = (T)ce_sinpi(k, 2 * N);
            X[k] = cph * Vr + sph * Vi;
            if constexpr (k >= 1 && k < M) X[N - k] = sph * Vr - cph * Vi;
        });
    }

    // x = N * DCT2^{-1}(X).
    __device__ __forceinline__ static void inverse(const T (&X)[N], T (&x)[N])
    {
        // V_k = e^{i pi k/2N} (X_k - i X_{N-k}), k = 0..M (X_N = 0).
        T Vr[M + 1], Vi[M + 1];
        static_for<0, M + 1>([&](auto Ki) {
            constexpr int k = Ki;
            constexpr T c = (T)ce_cospi(k, 2 * N);
            constexpr T s = (T)ce_sinpi(k, 2 * N);
            const T xk = X[k];
            if constexpr (k == 0) {
                Vr[0] = xk;
                Vi[0] = T(0);
            } else {
                const T xn = X[N - k];
                Vr[k] = c * xk + s * xn;
                Vi[k] = s * xk - c * xn;
            }
        });
        // Undo the split: 2E_k = V_k + conj(V_{M-k}), 2O_k = (V_k - conj(V_{M-k})) e^{2 pi i k/N},
        // Z_k = E_k + i O_k, stored bit-reversed for the backward FFT.
        T zr[M], zi[M];
        static_for<0, M>([&](auto Ki) {
            constexpr int k = Ki;
            constexpr int p = bitrev(k, LOGM);
            const T a = Vr[k], b = Vi[k], c = Vr[M - k], d = -Vi[M - k];
            const T Er = a + c, Ei = b + d;
            const T pr = a - c, pi = b - d;
            constexpr T wr = (T)ce_cospi(2 * k, N);
            constexpr T wi = (T)ce_sinpi(2 * k, N);
            const T Or = wr * pr - wi * pi;
            const T Oi = wr * pi + wi * pr;
            zr[p] = Er - Oi;
            zi[p] = Ei + Or;
        });
        fft<+1>(zr, zi);
        static_for<0, M>([&](auto Mi) {
            constexpr int m = Mi;
            x[vsrc(2 * m)] = zr[m];
            x[vsrc(2 * m + 1)] = zi[m];
        });
    }
};

}  // namespace cil
