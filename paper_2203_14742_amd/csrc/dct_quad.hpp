// Length-N DCT-II and its inverse on one line spread over a quad of lanes.
//
// Same mathematics as dct_reg.hpp (Makhoul's reduction to a length-N real DFT,
// which is a length-M = N/2 complex FFT plus a split step), but the complex
// FFT is taken in four steps, M = P x 4 with P = N/8:
//   z_m, m = 4 m1 + q, lives in lane q of the quad (P values);
//   each lane takes a P-point FFT over m1 (registers, literal twiddles),
//   multiplies by W_M^(q k1), and the quad finishes with a 4-point DFT across
//   its lanes (two radix-2 stages exchanging registers by DPP quad permutes).
// Lane q then holds Z_k for k = k1 + P k2(q), k2(q) = (q >> 1) + 2 (q & 1),
// k1 = 0..P-1; the split step pairs k with M - k, found in lane q ^ 3 (for
// k1 = 0 in lane q or q ^ 1).  The inverse runs the same steps backwards.
// A quad therefore moves a line with a quarter of the registers and work per
// lane of the one-lane transform, which gives a solve four times the waves.
//
// Scaling (folded into the spectral divisor): forward = 2 DCT2,
// inverse = N DCT2^{-1}.  Input and output live in LDS, addressed by the
// caller's functors; a line is updated in place by its own quad.
#pragma once

#include "cil_internal.hpp"

namespace cil {

// quad_perm controls: lane q reads lane q ^ 1, q ^ 2, q ^ 3 of its quad
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_XOR3 = 0x1B;

template <int CTRL>
__device__ __forceinline__ float quad_swap(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <typename T, int N>
struct QuadLine {
    static constexpr int M = N / 2;
    static constexpr int P = M / 4;
    static constexpr int LOGP = ilog2(P);
    static_assert(P >= 2 && (1 << LOGP) == P, "N must be a power of two >= 16");

    // Per-lane constants, computed once per kernel.
    struct Lane {
        int q, k2;
        T tw_r[P], tw_i[P];   // W_M^(q k1) = exp(-2 pi i q k1 / M)
        T al_r, al_i;         // exp(-2 pi i P k2 / N)
        T be_r, be_i;         // exp(-i pi P k2 / (2N))
    };

    __device__ static void init(Lane &L, int q)
    {
        L.q = q;
        L.k2 = (q >> 1) + 2 * (q & 1);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) {
            double s, c;
            sincospi(-2.0 * q * k1 / (double)M, &s, &c);
            L.tw_r[k1] = (T)c;
            L.tw_i[k1] = (T)s;
        }
        double s, c;
        sincospi(-2.0 * P * L.k2 / (double)N, &s, &c);
        L.al_r = (T)c;
        L.al_i = (T)s;
        sincospi(-(double)P * L.k2 / (2.0 * N), &s, &c);
        L.be_r = (T)c;
        L.be_i = (T)s;
    }

    // index of the input element that lands at position j of the reordering
    __device__ static int vsrc(int j) { return j < M ? 2 * j : 2 * (N - 1 - j) + 1; }

    template <int SIGN>
    __device__ __forceinline__ static void fftP(T (&re)[P], T (&im)[P])
    {
        static_for<1, LOGP + 1>([&](auto S) {
            constexpr int m = 1 << S;
            constexpr int h = m / 2;
            static_for<0, P / m>([&](auto Bk) {
                constexpr int k0 = Bk * m;
                static_for<0, h>([&](auto J) {
                    constexpr int j = J;
                    constexpr int a = k0 + j, b = a + h;
                    T tr, ti;
                    if constexpr (j == 0) {
                        tr = re[b];
                        ti = im[b];
                    } else if constexpr (4 * j == m) {
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

    // 4-point DFT across the quad.  Forward: lane q enters with Y_q, leaves
    // with the output index k2(q).  Backward: lane q enters holding index
    // k2(q) and leaves with output index q.
    __device__ __forceinline__ static void cross_fwd(const Lane &L, T (&re)[P], T (&im)[P])
    {
        const T s1 = (L.q >> 1) ? T(-1) : T(1);
        const T s2 = (L.q & 1) ? T(-1) : T(1);
        const bool rot = (L.q == 3);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const T pr = quad_swap<DPP_XOR2>(re[k]), pi = quad_swap<DPP_XOR2>(im[k]);
            T ar = pr + s1 * re[k], ai = pi + s1 * im[k];
            const T tr = rot ? ai : ar, ti = rot ? -ar : ai;      // times -i on lane 3
            const T qr = quad_swap<DPP_XOR1>(tr), qi = quad_swap<DPP_XOR1>(ti);
            re[k] = qr + s2 * tr;
            im[k] = qi + s2 * ti;
        }
    }
    __device__ __forceinline__ static void cross_bwd(const Lane &L, T (&re)[P], T (&im)[P])
    {
        const T s1 = (L.q & 1) ? T(-1) : T(1);
        const T s2 = (L.q >> 1) ? T(-1) : T(1);
        const bool rot = (L.q == 3);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const T pr = quad_swap<DPP_XOR1>(re[k]), pi = quad_swap<DPP_XOR1>(im[k]);
            T cr = pr + s1 * re[k], ci = pi + s1 * im[k];
            const T tr = rot ? -ci : cr, ti = rot ? cr : ci;      // times +i on lane 3
            const T qr = quad_swap<DPP_XOR2>(tr), qi = quad_swap<DPP_XOR2>(ti);
            re[k] = qr + s2 * tr;
            im[k] = qi + s2 * ti;
        }
    }

    // Forward: gathered line -> X_k (k = k1 + P k2) and X_{N-k}, written by st(index, value).
    template <typename LD, typename ST>
    __device__ __forceinline__ static void forward(const Lane &L, LD &&ld, ST &&st)
    {
        T zr[P], zi[P];
        static_for<0, P>([&](auto Mi) {
            constexpr int m1 = Mi;
            constexpr int p = bitrev(m1, LOGP);
            const int j = 2 * (4 * m1 + L.q);
            zr[p] = ld(vsrc(j));
            zi[p] = ld(vsrc(j + 1));
        });
        forward_from(L, zr, zi, st);
    }

    // Same, from values already in registers (bit-reversed m1 order).
    template <typename ST>
    __device__ __forceinline__ static void forward_from(const Lane &L, T (&zr)[P], T (&zi)[P], ST &&st)
    {
        fftP<-1>(zr, zi);
#pragma unroll
        for (int k1 = 1; k1 < P; ++k1) {
            const T r = zr[k1] * L.tw_r[k1] - zi[k1] * L.tw_i[k1];
            const T i = zr[k1] * L.tw_i[k1] + zi[k1] * L.tw_r[k1];
            zr[k1] = r;
            zi[k1] = i;
        }
        cross_fwd(L, zr, zi);
        const int kb = P * L.k2;
        static_for<0, P>([&](auto Ki) {
            constexpr int k1 = Ki;
            // partner conj(Z_{M-k}): lane q ^ 3 at P - k1; for k1 = 0 lane q (q < 2) or q ^ 1
            T c, d;
            if constexpr (k1 == 0) {
                const T sr = quad_swap<DPP_XOR1>(zr[0]), si = quad_swap<DPP_XOR1>(zi[0]);
                c = L.q < 2 ? zr[0] : sr;
                d = L.q < 2 ? -zi[0] : -si;
            } else {
                c = quad_swap<DPP_XOR3>(zr[P - k1]);
                d = -quad_swap<DPP_XOR3>(zi[P - k1]);
            }
            const T a = zr[k1], b = zi[k1];
            const T Er = a + c, Ei = b + d, Or = b - d, Oi = c - a;
            // w = exp(-2 pi i k / N) = lit(k1) * alpha;  ph = exp(-i pi k / 2N) = lit'(k1) * beta
            constexpr T l1r = (T)ce_cospi(2 * k1, N), l1i = (T)(-ce_sinpi(2 * k1, N));
            constexpr T l2r = (T)ce_cospi(k1, 2 * N), l2i = (T)(-ce_sinpi(k1, 2 * N));
            const T wr = l1r * L.al_r - l1i * L.al_i, wi = l1r * L.al_i + l1i * L.al_r;
            const T hr = l2r * L.be_r - l2i * L.be_i, hi = l2r * L.be_i + l2i * L.be_r;
            const T Vr = Er + (wr * Or - wi * Oi), Vi = Ei + (wr * Oi + wi * Or);
            const int k = k1 + kb;
            st(k, hr * Vr - hi * Vi);
            if (k != 0) st(N - k, -(hr * Vi + hi * Vr));
            if constexpr (k1 == 0) {
                if (L.q == 0) {      // k = M from the same pair: w = -1, ph = exp(-i pi / 4)
                    constexpr T c4 = (T)ce_cospi(1, 4);
                    const T Ur = Er - Or, Ui = Ei - Oi;
                    st(M, c4 * (Ur + Ui));
                }
            }
        });
    }

    // Backward: reads X at k, N-k, M-k, M+k through ld; writes the line through st.
    template <typename LD, typename ST>
    __device__ __forceinline__ static void inverse(const Lane &L, LD &&ld, ST &&st)
    {
        T zr[P], zi[P];
        const int kb = P * L.k2;
        static_for<0, P>([&](auto Ki) {
            constexpr int k1 = Ki;
            const int k = k1 + kb;
            const T xk = ld(k), xn = (k == 0) ? T(0) : ld(N - k);
            const T ym = ld(M - k), yp = ld(M + k);         // X_{M-k}, X_{N-(M-k)} (both X_M at k = 0)
            build_z_c<k1>(L, xk, xn, ym, yp, zr, zi);
        });
        inverse_from(L, zr, zi, st);
    }

    // Z_k for one k1 from X_k, X_{N-k}, X_{M-k}, X_{M+k}; stored bit-reversed.
    template <int K1>
    __device__ __forceinline__ static void build_z_c(const Lane &L, T xk, T xn, T ym, T yp, T (&zr)[P], T (&zi)[P])
    {
        // ph = exp(-i pi k/2N); V_k = conj(ph) (X_k - i X_{N-k});
        // V_{M-k} = exp(i pi M/2N) exp(-i pi k/2N) (X_{M-k} - i X_{M+k}) = e^{i pi/4} ph (..)
        constexpr T l2r = (T)ce_cospi(K1, 2 * N), l2i = (T)(-ce_sinpi(K1, 2 * N));
        constexpr T l1r = (T)ce_cospi(2 * K1, N), l1i = (T)(-ce_sinpi(2 * K1, N));
        constexpr T c4 = (T)ce_cospi(1, 4);
        const T hr = l2r * L.be_r - l2i * L.be_i, hi = l2r * L.be_i + l2i * L.be_r;   // ph
        const T wr = l1r * L.al_r - l1i * L.al_i, wi = l1r * L.al_i + l1i * L.al_r;   // w = exp(-2 pi i k/N)
        // V_k = (hr - i hi)(xk - i xn)
        const T ar = hr * xk - hi * xn, ai = -(hr * xn + hi * xk);
        // g = e^{i pi/4} ph = c4 (1 + i)(hr + i hi)
        const T gr = c4 * (hr - hi), gi = c4 * (hr + hi);
        // V_{M-k} = g (ym - i yp); c + i d = conj(V_{M-k})
        const T vr = gr * ym + gi * yp, vi = gi * ym - gr * yp;
        const T c = vr, d = -vi;
        const T Er = ar + c, Ei = ai + d;
        const T pr = ar - c, pi = ai - d;
        // O = (p) conj(w)
        const T Or = pr * wr + pi * wi, Oi = pi * wr - pr * wi;
        constexpr int p = bitrev(K1, LOGP);
        zr[p] = Er - Oi;
        zi[p] = Ei + Or;
    }

    template <typename ST>
    __device__ __forceinline__ static void inverse_from(const Lane &L, T (&zr)[P], T (&zi)[P], ST &&st)
    {
        // zr/zi arrive bit-reversed in k1; the cross-lane stage works elementwise,
        // the lane twiddle needs the natural index
        cross_bwd(L, zr, zi);
        static_for<1, P>([&](auto Ki) {
            constexpr int k1 = Ki;
            constexpr int p = bitrev(k1, LOGP);
            const T r = zr[p] * L.tw_r[k1] + zi[p] * L.tw_i[k1];     // conj twiddle
            const T i = zi[p] * L.tw_r[k1] - zr[p] * L.tw_i[k1];
            zr[p] = r;
            zi[p] = i;
        });
        fftP<+1>(zr, zi);
        static_for<0, P>([&](auto Mi) {
            constexpr int m1 = Mi;
            const int j = 2 * (4 * m1 + L.q);
            st(vsrc(j), zr[m1]);
            st(vsrc(j + 1), zi[m1]);
        });
    }
};

}  // namespace cil
