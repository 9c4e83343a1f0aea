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
// inverse = N DCT2^{-1}.  Input and output are the lanes' registers: line
// values in the order the four-step split fixes (the caller moves them to and
// from LDS or HBM), spectral values as the pairs (X_k, X_{N-k}) a lane's own
// split step yields, so a forward transform, a pointwise spectral operation
// and an inverse chain without any data leaving the quad.
#pragma once

#include "cil_internal.hpp"

namespace cil {

// DPP controls.  quad_perm: lane q reads lane q ^ 1, q ^ 2, q ^ 3 of its quad;
// row_half_mirror: lane i reads lane 7 - i of its group of eight.  Every
// source lane of these patterns exists, so bound_ctrl (zero for a missing
// source) never acts; it is set because it lets the compiler fold a move into
// the VOP2 instruction that consumes it (v_add_f32_dpp and the like).
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_XOR3 = 0x1B, DPP_HALF_MIRROR = 0x141;

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// v[k] += c * (v[k] of the quad partner CTRL selects), for every k: a
// radix-2 stage across the quad with a lane sign c.  FP32: one
// v_fmac_f32_dpp per value, which the compiler does not form from a move and
// a multiply-add by itself, all in one asm block behind one s_nop: a DPP read
// of a VGPR needs two wait states after a VALU write of it, the hazard check
// does not look inside asm, and within the block every read is of a value
// written before it.  FP64: a move and a multiply-add per value.  Either way
// one rounding of v + c partner, as the two-instruction form.
#define CIL_QP1 "quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
#define CIL_QP2 "quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
#define CIL_QF(i, c, qp) "v_fmac_f32_dpp %" #i ", %" #i ", %" #c " " qp
#define CIL_QF4(a, b, d, e, c, qp) CIL_QF(a, c, qp) CIL_QF(b, c, qp) CIL_QF(d, c, qp) CIL_QF(e, c, qp)

template <int QP, int P>
__device__ __forceinline__ void quad_fmac_all_f32(float (&v)[P], float c)
{
    static_assert(QP == 1 || QP == 2, "quad_fmac_all: xor-1 or xor-2 partner");
    if constexpr (P == 4) {
        if constexpr (QP == 1)
            asm("s_nop 1\n\t" CIL_QF4(0, 1, 2, 3, 4, CIL_QP1) : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]) : "v"(c));
        else
            asm("s_nop 1\n\t" CIL_QF4(0, 1, 2, 3, 4, CIL_QP2) : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]) : "v"(c));
    } else if constexpr (P == 8) {
        if constexpr (QP == 1)
            asm("s_nop 1\n\t" CIL_QF4(0, 1, 2, 3, 8, CIL_QP1) CIL_QF4(4, 5, 6, 7, 8, CIL_QP1)
                : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7])
                : "v"(c));
        else
            asm("s_nop 1\n\t" CIL_QF4(0, 1, 2, 3, 8, CIL_QP2) CIL_QF4(4, 5, 6, 7, 8, CIL_QP2)
                : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7])
                : "v"(c));
    } else if constexpr (P == 16) {
        if constexpr (QP == 1)
            asm("s_nop 1\n\t" CIL_QF4(0, 1, 2, 3, 16, CIL_QP1) CIL_QF4(4, 5, 6, 7, 16, CIL_QP1)
                    CIL_QF4(8, 9, 10, 11, 16, CIL_QP1) CIL_QF4(12, 13, 14, 15, 16, CIL_QP1)
                : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7]),
                  "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]), "+v"(v[14]), "+v"(v[15])
                : "v"(c));
        else
            asm("s_nop 1\n\t" CIL_QF4(0, 1, 2, 3, 16, CIL_QP2) CIL_QF4(4, 5, 6, 7, 16, CIL_QP2)
                    CIL_QF4(8, 9, 10, 11, 16, CIL_QP2) CIL_QF4(12, 13, 14, 15, 16, CIL_QP2)
                : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7]),
                  "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]), "+v"(v[14]), "+v"(v[15])
                : "v"(c));
    } else {
        static_assert(P == 4 || P == 8 || P == 16, "quad_fmac_all: P = 4, 8 or 16");
    }
}

template <int QP, typename T, int P>
__device__ __forceinline__ void quad_fmac_all(T (&v)[P], T c)
{
    if constexpr (sizeof(T) == 4) {
        quad_fmac_all_f32<QP, P>(v, c);
    } else {
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = fma(dpp_mov<QP == 1 ? DPP_XOR1 : DPP_XOR2>(v[k]), c, v[k]);
    }
}

#undef CIL_QF4
#undef CIL_QF
#undef CIL_QP2
#undef CIL_QP1

// CT >= 1: the split step's twiddles w_k and ph_k (k = k1 + P k2) are held
// per lane in registers (4P more), one complex product each; CT = 2 also
// e^{i pi/4} ph_k (2P more).  Otherwise each is a lane constant times a
// literal: two products and no register.
template <typename T, int N, int CT = 0>
struct QuadLine {
    static constexpr int M = N / 2;
    static constexpr int P = M / 4;
    static constexpr int LOGP = ilog2(P);
    static constexpr int PC = CT >= 1 ? P : 1, PG = CT >= 2 ? P : 1;
    static_assert(P >= 2 && (1 << LOGP) == P, "N must be a power of two >= 16");

    // Per-lane constants, computed once per kernel.
    struct Lane {
        int q, k2;
        T tw_r[P], tw_i[P];   // rho W_M^(q k1), W_M^(q k1) = exp(-2 pi i q k1 / M), for k1 >= 1
        T al_r, al_i;         // exp(-2 pi i P k2 / N)
        T be_r, be_i;         // exp(-i pi P k2 / (2N))
        T w_r[PC], w_i[PC];   // CT: w_k = exp(-2 pi i k / N)
        T ph_r[PC], ph_i[PC]; // CT: ph_k = exp(-i pi k / 2N)
        T g_r[PG], g_i[PG];   // CT = 2: e^{i pi/4} ph_k = exp(-i pi (k - N/2) / 2N)
    };

    // The lane constants, selected from compile-time values (exact to the
    // last bit of T, no run-time trigonometry).
    __device__ static void init(Lane &L, int q)
    {
        L.q = q;
        L.k2 = (q >> 1) + 2 * (q & 1);
        static_for<0, P>([&](auto Ki) {
            constexpr int k1 = Ki;
            // rho W_M^(q k1) for q = 0..3, rho = rho(q) of the cross-lane stage
            constexpr T r1 = (T)ce_cospi(2 * k1, M), i1 = (T)(-ce_sinpi(2 * k1, M));
            constexpr T r2 = (T)ce_cospi(4 * k1, M), i2 = (T)(-ce_sinpi(4 * k1, M));
            constexpr T r3 = (T)ce_cospi(6 * k1, M), i3 = (T)(-ce_sinpi(6 * k1, M));
            L.tw_r[k1] = q == 0 ? T(1) : (q == 1 ? -r1 : (q == 2 ? -r2 : r3));
            L.tw_i[k1] = q == 0 ? T(0) : (q == 1 ? -i1 : (q == 2 ? -i2 : i3));
        });
        // alpha = exp(-2 pi i P k2 / N), beta = exp(-i pi P k2 / 2N) for k2 = 0..3
        const int k2 = L.k2;
        constexpr T a1r = (T)ce_cospi(2 * P, N), a1i = (T)(-ce_sinpi(2 * P, N));
        constexpr T a2r = (T)ce_cospi(4 * P, N), a2i = (T)(-ce_sinpi(4 * P, N));
        constexpr T a3r = (T)ce_cospi(6 * P, N), a3i = (T)(-ce_sinpi(6 * P, N));
        constexpr T b1r = (T)ce_cospi(P, 2 * N), b1i = (T)(-ce_sinpi(P, 2 * N));
        constexpr T b2r = (T)ce_cospi(2 * P, 2 * N), b2i = (T)(-ce_sinpi(2 * P, 2 * N));
        constexpr T b3r = (T)ce_cospi(3 * P, 2 * N), b3i = (T)(-ce_sinpi(3 * P, 2 * N));
        L.al_r = k2 == 0 ? T(1) : (k2 == 1 ? a1r : (k2 == 2 ? a2r : a3r));
        L.al_i = k2 == 0 ? T(0) : (k2 == 1 ? a1i : (k2 == 2 ? a2i : a3i));
        L.be_r = k2 == 0 ? T(1) : (k2 == 1 ? b1r : (k2 == 2 ? b2r : b3r));
        L.be_i = k2 == 0 ? T(0) : (k2 == 1 ? b1i : (k2 == 2 ? b2i : b3i));
        if constexpr (CT >= 1) {
            // each rounded once from its exact value, selected by k2
            static_for<0, P>([&](auto Ki) {
                constexpr int k1 = Ki;
                auto sel = [&](auto f0, auto f1, auto f2, auto f3) { return k2 == 0 ? f0 : (k2 == 1 ? f1 : (k2 == 2 ? f2 : f3)); };
                L.w_r[k1] = sel((T)ce_cospi(2 * k1, N), (T)ce_cospi(2 * (k1 + P), N), (T)ce_cospi(2 * (k1 + 2 * P), N),
                                (T)ce_cospi(2 * (k1 + 3 * P), N));
                L.w_i[k1] = sel((T)-ce_sinpi(2 * k1, N), (T)-ce_sinpi(2 * (k1 + P), N),
                                (T)-ce_sinpi(2 * (k1 + 2 * P), N), (T)-ce_sinpi(2 * (k1 + 3 * P), N));
                L.ph_r[k1] = sel((T)ce_cospi(k1, 2 * N), (T)ce_cospi(k1 + P, 2 * N), (T)ce_cospi(k1 + 2 * P, 2 * N),
                                 (T)ce_cospi(k1 + 3 * P, 2 * N));
                L.ph_i[k1] = sel((T)-ce_sinpi(k1, 2 * N), (T)-ce_sinpi(k1 + P, 2 * N), (T)-ce_sinpi(k1 + 2 * P, 2 * N),
                                 (T)-ce_sinpi(k1 + 3 * P, 2 * N));
                constexpr int h = N / 2;
                if constexpr (CT >= 2) {
                L.g_r[k1] = sel((T)ce_cospi(k1 - h, 2 * N), (T)ce_cospi(k1 + P - h, 2 * N),
                                (T)ce_cospi(k1 + 2 * P - h, 2 * N), (T)ce_cospi(k1 + 3 * P - h, 2 * N));
                L.g_i[k1] = sel((T)-ce_sinpi(k1 - h, 2 * N), (T)-ce_sinpi(k1 + P - h, 2 * N),
                                (T)-ce_sinpi(k1 + 2 * P - h, 2 * N), (T)-ce_sinpi(k1 + 3 * P - h, 2 * N));
                }
            });
        }
    }

    // index of the input element that lands at position j of the reordering
    __device__ static int vsrc(int j) { return j < M ? 2 * j : 2 * (N - 1 - j) + 1; }

    // Line position of lane q's value h (0: real part, 1: imaginary part) of
    // pair m1, i.e. vsrc(2 (4 m1 + q) + h), split so that the lane-dependent
    // part is one base per half: pairs m1 < P/2 lie at 4q + 16 m1 + 2h, the
    // others at (2N - 1 - 4q) - 16 m1 - 2h.
    template <int m1, int h>
    __device__ static constexpr int pos_off() { return m1 < P / 2 ? 16 * m1 + 2 * h : -(16 * m1 + 2 * h); }
    template <int m1>
    __device__ static int pos_base(int q) { return m1 < P / 2 ? 4 * q : 2 * N - 1 - 4 * q; }

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
                        // a + w b as multiply-add chains into a, then a - w b as
                        // 2 a - (a + w b): three instructions per part instead of
                        // four, within one rounding of the sum
                        constexpr T wr = (T)ce_cospi(2 * j, m);
                        constexpr T wi = (T)(SIGN * ce_sinpi(2 * j, m));
                        const T ar = re[a], ai = im[a];
                        re[a] = fma(wr, re[b], fma(-wi, im[b], ar));
                        im[a] = fma(wr, im[b], fma(wi, re[b], ai));
                        re[b] = fma(T(2), ar, -re[a]);
                        im[b] = fma(T(2), ai, -im[a]);
                        return;
                    }
                    re[b] = re[a] - tr;
                    im[b] = im[a] - ti;
                    re[a] = re[a] + tr;
                    im[a] = im[a] + ti;
                });
            });
        });
    }

    // 4-point DFT across the quad.  Forward: lane q enters with rho(q) Y_q and
    // leaves with the output index k2(q).  Backward: lane q enters holding
    // index k2(q) and leaves with rho(q) times output index q.  rho = +1, -1,
    // -1, +1 on q = 0..3 is the sign that lets every radix-2 stage be
    // own + c(q) partner (one quad_fmac: the lane's own value with coefficient
    // 1, the partner's with a lane sign), and it is folded into the lane
    // twiddles around the stage (and applied to k1 = 0, which has none).
    // Forward: stage 1 (partner q ^ 2) c = -1, -1, +1, +1; lane 3 times -i;
    // stage 2 (partner q ^ 1) c = -1, +1, -1, +1.  Backward: stage 1 (q ^ 1)
    // c = +1, -1, +1, -1; lane 3 times +i; stage 2 (q ^ 2) c = +1, +1, -1, -1.
    // Sign flips are exact, so the values equal those of the plain
    // sum-and-difference butterflies bit for bit.
    __device__ __forceinline__ static T rho(const Lane &L) { return ((L.q >> 1) ^ (L.q & 1)) ? T(-1) : T(1); }
    __device__ __forceinline__ static void cross_fwd(const Lane &L, T (&re)[P], T (&im)[P])
    {
        const T c1 = (L.q >> 1) ? T(1) : T(-1);
        const T c2 = (L.q & 1) ? T(1) : T(-1);
        const bool rot = (L.q == 3);
        quad_fmac_all<2>(re, c1);
        quad_fmac_all<2>(im, c1);
#pragma unroll
        for (int k = 0; k < P; ++k) {                             // times -i on lane 3
            const T ar = re[k], ai = im[k];
            re[k] = rot ? ai : ar;
            im[k] = rot ? -ar : ai;
        }
        quad_fmac_all<1>(re, c2);
        quad_fmac_all<1>(im, c2);
    }
    __device__ __forceinline__ static void cross_bwd(const Lane &L, T (&re)[P], T (&im)[P])
    {
        const T c1 = (L.q & 1) ? T(-1) : T(1);
        const T c2 = (L.q >> 1) ? T(-1) : T(1);
        const bool rot = (L.q == 3);
        quad_fmac_all<1>(re, c1);
        quad_fmac_all<1>(im, c1);
#pragma unroll
        for (int k = 0; k < P; ++k) {                             // times +i on lane 3
            const T cr = re[k], ci = im[k];
            re[k] = rot ? -ci : cr;
            im[k] = rot ? cr : ci;
        }
        quad_fmac_all<2>(re, c2);
        quad_fmac_all<2>(im, c2);
    }

    // Forward, from the lane's 2P line values (bit-reversed m1 order: zr[bitrev(m1)]
    // at position vsrc(2(4 m1 + q)), zi[...] at the next one) to its spectral
    // values: xa[k1] = X_k, xb[k1] = X_{N-k}, k = k1 + P k2 (xb = 0 where k = 0),
    // and xm = X_M on lane q = 0.  zr/zi are destroyed.
    __device__ __forceinline__ static void forward_regs(const Lane &L, T (&zr)[P], T (&zi)[P], T (&xa)[P],
                                                        T (&xb)[P], T &xm)
    {
        fftP<-1>(zr, zi);
        zr[0] *= rho(L);
        zi[0] *= rho(L);
#pragma unroll
        for (int k1 = 1; k1 < P; ++k1) {
            const T r = zr[k1] * L.tw_r[k1] - zi[k1] * L.tw_i[k1];
            const T i = zr[k1] * L.tw_i[k1] + zi[k1] * L.tw_r[k1];
            zr[k1] = r;
            zi[k1] = i;
        }
        cross_fwd(L, zr, zi);
        // k1 and P - k1 are each other's partners: take them together so that
        // both Z values die at once
        static_for<0, P>([&](auto Ji) {
            constexpr int J = Ji;
            constexpr int k1 = (J == 0) ? 0 : ((J & 1) ? (J + 1) / 2 : P - J / 2);
            // partner conj(Z_{M-k}): lane q ^ 3 at P - k1; for k1 = 0 lane q (q < 2) or q ^ 1
            T c, d;
            if constexpr (k1 == 0) {
                const T sr = dpp_mov<DPP_XOR1>(zr[0]), si = dpp_mov<DPP_XOR1>(zi[0]);
                c = L.q < 2 ? zr[0] : sr;
                d = L.q < 2 ? -zi[0] : -si;
            } else {
                c = dpp_mov<DPP_XOR3>(zr[P - k1]);
                d = -dpp_mov<DPP_XOR3>(zi[P - k1]);
            }
            const T a = zr[k1], b = zi[k1];
            const T Er = a + c, Ei = b + d, Or = b - d, Oi = c - a;
            // V = E + w O with w = exp(-2 pi i k / N) = lit1(k1) alpha, and
            // X_k - i X_{N-k} = ph V with ph = exp(-i pi k / 2N) = lit2(k1) beta.
            // The lane constant multiplies the data first, then the literal:
            // the same operation count as forming w and ph, and no per-k1 lane
            // twiddles that the compiler could precompute and keep live.
            if constexpr (CT >= 1) {
                const T Vr = fma(L.w_r[k1], Or, fma(-L.w_i[k1], Oi, Er));
                const T Vi = fma(L.w_r[k1], Oi, fma(L.w_i[k1], Or, Ei));
                xa[k1] = L.ph_r[k1] * Vr - L.ph_i[k1] * Vi;
                xb[k1] = -(L.ph_r[k1] * Vi + L.ph_i[k1] * Vr);
            } else {
                constexpr T l1r = (T)ce_cospi(2 * k1, N), l1i = (T)(-ce_sinpi(2 * k1, N));
                constexpr T l2r = (T)ce_cospi(k1, 2 * N), l2i = (T)(-ce_sinpi(k1, 2 * N));
                const T ar = L.al_r * Or - L.al_i * Oi, ai = L.al_r * Oi + L.al_i * Or;      // alpha O
                const T Vr = fma(l1r, ar, fma(-l1i, ai, Er)), Vi = fma(l1r, ai, fma(l1i, ar, Ei));
                const T br = L.be_r * Vr - L.be_i * Vi, bi = L.be_r * Vi + L.be_i * Vr;      // beta V
                xa[k1] = l2r * br - l2i * bi;
                xb[k1] = -(l2r * bi + l2i * br);
            }
            if constexpr (k1 == 0) {
                // k = M from the same pair on lane 0: w = -1, ph = exp(-i pi / 4)
                constexpr T c4 = (T)ce_cospi(1, 4);
                xm = c4 * ((Er - Or) + (Ei - Oi));
                if (L.q == 0) xb[0] = T(0);
            }
        });
    }

    // Forward as far as the split step's V_k = E_k + w_k O_k (k = k1 + P k2),
    // with X_k - i X_{N-k} = ph_k V_k; xm = X_M on lane q = 0 as in forward_regs.
    __device__ __forceinline__ static void forward_v(const Lane &L, T (&zr)[P], T (&zi)[P], T (&vr)[P], T (&vi)[P],
                                                     T &xm)
    {
        fftP<-1>(zr, zi);
        zr[0] *= rho(L);
        zi[0] *= rho(L);
#pragma unroll
        for (int k1 = 1; k1 < P; ++k1) {
            const T r = zr[k1] * L.tw_r[k1] - zi[k1] * L.tw_i[k1];
            const T i = zr[k1] * L.tw_i[k1] + zi[k1] * L.tw_r[k1];
            zr[k1] = r;
            zi[k1] = i;
        }
        cross_fwd(L, zr, zi);
        static_for<0, P>([&](auto Ji) {
            constexpr int J = Ji;
            constexpr int k1 = (J == 0) ? 0 : ((J & 1) ? (J + 1) / 2 : P - J / 2);
            T c, d;
            if constexpr (k1 == 0) {
                const T sr = dpp_mov<DPP_XOR1>(zr[0]), si = dpp_mov<DPP_XOR1>(zi[0]);
                c = L.q < 2 ? zr[0] : sr;
                d = L.q < 2 ? -zi[0] : -si;
            } else {
                c = dpp_mov<DPP_XOR3>(zr[P - k1]);
                d = -dpp_mov<DPP_XOR3>(zi[P - k1]);
            }
            const T a = zr[k1], b = zi[k1];
            const T Er = a + c, Ei = b + d, Or = b - d, Oi = c - a;
            if constexpr (CT >= 1) {
                vr[k1] = fma(L.w_r[k1], Or, fma(-L.w_i[k1], Oi, Er));
                vi[k1] = fma(L.w_r[k1], Oi, fma(L.w_i[k1], Or, Ei));
            } else {
                constexpr T l1r = (T)ce_cospi(2 * k1, N), l1i = (T)(-ce_sinpi(2 * k1, N));
                const T ar = L.al_r * Or - L.al_i * Oi, ai = L.al_r * Oi + L.al_i * Or;      // alpha O
                vr[k1] = fma(l1r, ar, fma(-l1i, ai, Er));
                vi[k1] = fma(l1r, ai, fma(l1i, ar, Ei));
            }
            if constexpr (k1 == 0) {
                constexpr T c4 = (T)ce_cospi(1, 4);
                xm = c4 * ((Er - Or) + (Ei - Oi));
            }
        });
    }

    // Inverse from V'_k (as forward_v leaves them, after a spectral operator)
    // and X'_M on lane 0: Z_k = E + i O with E = V'_k + conj(V'_{M-k}),
    // O = (V'_k - conj(V'_{M-k})) conj(w_k); V'_{M-k} comes from lane q ^ 3 at
    // P - k1 (k1 = 0: the lane itself, its xor-1 neighbour, or V'_M = sqrt(2) X'_M).
    __device__ __forceinline__ static void inverse_v(const Lane &L, const T (&vr)[P], const T (&vi)[P], T xm,
                                                     T (&zr)[P], T (&zi)[P])
    {
        static_for<0, P>([&](auto Ji) {
            constexpr int J = Ji;
            constexpr int k1 = (J == 0) ? 0 : ((J & 1) ? (J + 1) / 2 : P - J / 2);
            T mr, mi;     // V'_{M-k}
            if constexpr (k1 == 0) {
                constexpr T s2 = (T)1.4142135623730950488;
                const T sr = dpp_mov<DPP_XOR1>(vr[0]), si = dpp_mov<DPP_XOR1>(vi[0]);
                mr = L.q == 0 ? s2 * xm : (L.q == 1 ? vr[0] : sr);
                mi = L.q == 0 ? T(0) : (L.q == 1 ? vi[0] : si);
            } else {
                mr = dpp_mov<DPP_XOR3>(vr[P - k1]);
                mi = dpp_mov<DPP_XOR3>(vi[P - k1]);
            }
            const T Er = vr[k1] + mr, Ei = vi[k1] - mi;
            const T pr = vr[k1] - mr, pi = vi[k1] + mi;
            // Z = E + i O, O = p conj(w): each part one chain of multiply-adds into E
            constexpr int p = bitrev(k1, LOGP);
            if constexpr (CT >= 1) {
                zr[p] = fma(-pi, L.w_r[k1], fma(pr, L.w_i[k1], Er));
                zi[p] = fma(pr, L.w_r[k1], fma(pi, L.w_i[k1], Ei));
            } else {
                constexpr T l1r = (T)ce_cospi(2 * k1, N), l1i = (T)(-ce_sinpi(2 * k1, N));
                const T t3r = pr * L.al_r + pi * L.al_i, t3i = pi * L.al_r - pr * L.al_i;   // p conj(alpha)
                zr[p] = fma(-l1r, t3i, fma(l1i, t3r, Er));
                zi[p] = fma(l1r, t3r, fma(l1i, t3i, Ei));
            }
        });
        inverse_core(L, zr, zi);
    }

    // Inverse, from the lane's spectral values (as forward_regs leaves them) to
    // its 2P line values in natural m1 order: zr[m1] at position
    // vsrc(2(4 m1 + q)), zi[m1] at the next.  The split step needs X_{M-k} and
    // X_{M+k} too, which lane q ^ 3 holds as its own pair at P - k1 (for
    // k1 = 0: lane q itself, its xor-1 neighbour, or X_M on lane 0).
    __device__ __forceinline__ static void inverse_regs(const Lane &L, const T (&xa)[P], const T (&xb)[P], T xm,
                                                        T (&zr)[P], T (&zi)[P])
    {
        static_for<0, P>([&](auto Ji) {          // partners k1, P - k1 together
            constexpr int J = Ji;
            constexpr int k1 = (J == 0) ? 0 : ((J & 1) ? (J + 1) / 2 : P - J / 2);
            T ym, yp;
            if constexpr (k1 == 0) {
                const T sa = dpp_mov<DPP_XOR1>(xa[0]), sb = dpp_mov<DPP_XOR1>(xb[0]);
                ym = L.q == 0 ? xm : (L.q == 1 ? xa[0] : sa);
                yp = L.q == 0 ? xm : (L.q == 1 ? xb[0] : sb);
            } else {
                ym = dpp_mov<DPP_XOR3>(xa[P - k1]);
                yp = dpp_mov<DPP_XOR3>(xb[P - k1]);
            }
            build_z_c<k1>(L, xa[k1], xb[k1], ym, yp, zr, zi);
        });
        inverse_core(L, zr, zi);
    }

    // Z_k for one k1 from X_k, X_{N-k}, X_{M-k}, X_{M+k}; stored bit-reversed.
    // ph = exp(-i pi k/2N) = lit2 beta, w = exp(-2 pi i k/N) = lit1 alpha;
    //   V_k     = conj(ph) (X_k - i X_{N-k}),
    //   V_{M-k} = e^{i pi/4} ph (X_{M-k} - i X_{M+k}),
    //   Z_k     = E + i O, E = V_k + conj(V_{M-k}), O = (V_k - conj(V_{M-k})) conj(w).
    // As in the forward, lane constants multiply data before literals.
    template <int K1>
    __device__ __forceinline__ static void build_z_c(const Lane &L, T xk, T xn, T ym, T yp, T (&zr)[P], T (&zi)[P])
    {
        if constexpr (CT >= 1) {
            // conj(ph) (xk - i xn); conj(g (ym - i yp)), g = e^{i pi/4} ph; O = p conj(w)
            const T ar = L.ph_r[K1] * xk - L.ph_i[K1] * xn, ai = -(L.ph_r[K1] * xn + L.ph_i[K1] * xk);
            // E = a + (c + i d), p = a - (c + i d): E by multiply-add chains into a, p as 2 a - E
            T Er, Ei;
            if constexpr (CT >= 2) {
                Er = fma(L.g_r[K1], ym, fma(L.g_i[K1], yp, ar));
                Ei = fma(L.g_r[K1], yp, fma(-L.g_i[K1], ym, ai));
            } else {                   // beta (ym - i yp), then e^{i pi/4} lit2, conjugated
                constexpr T l2r = (T)ce_cospi(K1, 2 * N), l2i = (T)(-ce_sinpi(K1, 2 * N));
                constexpr T c4 = (T)ce_cospi(1, 4);
                constexpr T gr = c4 * (l2r - l2i), gi = c4 * (l2r + l2i);
                const T t2r = L.be_r * ym + L.be_i * yp, t2i = L.be_i * ym - L.be_r * yp;
                Er = fma(gr, t2r, fma(-gi, t2i, ar));
                Ei = fma(-gr, t2i, fma(-gi, t2r, ai));
            }
            const T pr = fma(T(2), ar, -Er), pi = fma(T(2), ai, -Ei);
            constexpr int p = bitrev(K1, LOGP);          // Z = E + i p conj(w)
            zr[p] = fma(-pi, L.w_r[K1], fma(pr, L.w_i[K1], Er));
            zi[p] = fma(pr, L.w_r[K1], fma(pi, L.w_i[K1], Ei));
            return;
        }
        constexpr T l2r = (T)ce_cospi(K1, 2 * N), l2i = (T)(-ce_sinpi(K1, 2 * N));
        constexpr T l1r = (T)ce_cospi(2 * K1, N), l1i = (T)(-ce_sinpi(2 * K1, N));
        constexpr T c4 = (T)ce_cospi(1, 4);
        constexpr T gr = c4 * (l2r - l2i), gi = c4 * (l2r + l2i);     // e^{i pi/4} lit2
        // conj(beta) (xk - i xn), then conj(lit2)
        const T t1r = L.be_r * xk - L.be_i * xn, t1i = -(L.be_r * xn + L.be_i * xk);
        const T ar = l2r * t1r + l2i * t1i, ai = l2r * t1i - l2i * t1r;
        // beta (ym - i yp), then e^{i pi/4} lit2; c + i d = conj(V_{M-k})
        const T t2r = L.be_r * ym + L.be_i * yp, t2i = L.be_i * ym - L.be_r * yp;
        const T Er = fma(gr, t2r, fma(-gi, t2i, ar)), Ei = fma(-gr, t2i, fma(-gi, t2r, ai));
        const T pr = fma(T(2), ar, -Er), pi = fma(T(2), ai, -Ei);          // a - (c + i d)
        // O = p conj(alpha) conj(lit1)
        const T t3r = pr * L.al_r + pi * L.al_i, t3i = pi * L.al_r - pr * L.al_i;
        constexpr int p = bitrev(K1, LOGP);              // Z = E + i O
        zr[p] = fma(-l1r, t3i, fma(l1i, t3r, Er));
        zi[p] = fma(l1r, t3r, fma(l1i, t3i, Ei));
    }

    // zr/zi arrive bit-reversed in k1; the cross-lane stage works elementwise,
    // the lane twiddle needs the natural index.  Leaves natural m1 order.
    __device__ __forceinline__ static void inverse_core(const Lane &L, T (&zr)[P], T (&zi)[P])
    {
        cross_bwd(L, zr, zi);
        zr[0] *= rho(L);
        zi[0] *= rho(L);
        static_for<1, P>([&](auto Ki) {
            constexpr int k1 = Ki;
            constexpr int p = bitrev(k1, LOGP);
            const T r = zr[p] * L.tw_r[k1] + zi[p] * L.tw_i[k1];     // conj twiddle
            const T i = zi[p] * L.tw_r[k1] - zr[p] * L.tw_i[k1];
            zr[p] = r;
            zi[p] = i;
        });
        fftP<+1>(zr, zi);
    }
};

}  // namespace cil
