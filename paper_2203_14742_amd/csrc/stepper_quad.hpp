// The quad-lane persistent stepper (templates), instantiated per precision
// by stepper_quad_f32.hip and stepper_quad_f64.hip.
#pragma once

#include "dct_quad.hpp"
#include "stepper_common.hpp"

namespace cil {

// One solve of the quad variant (below), for one model.  SPL = species per
// lane: 2 (4N threads; quad g owns row/column g of both species) or 1 (8N
// threads; group g of eight lanes owns row/column g, species s = (t / 4) & 1,
// quad position q = t & 3 for v and 3 - (t & 3) for w, so that lane t ^ 7 -
// the DPP half-row mirror - holds the other species at the same points).
//
// The lane's values of u live in ur/ui (caller's registers): loaded from
// `state` first when LOAD, stored to `out` (element type TS, same layout) at
// the end.  `step` enters as the first step and leaves as the last; the
// return value is the status of the last evaluation (-1 if none ran).
//
// RF (refinement form, T = float): u = U + v with U in FP64 (u64, state
// layout) and the correction v in ur/ui.  One step of the same IMEX Euler
// iteration in these variables is
//     v' = S(v + dt (R + f(U + v) - f(U))),   R = f(U) + nu Lap U,
// S the diffusion solve: the transforms act on v, whose size is that of the
// motion since U was last set, so FP32 rounding stays proportional to it and
// the iteration has no FP32 floor.  R is formed in FP64 (five-point stencil
// with ghost copies, the Laplacian the DCT-II solve diagonalises) and the
// reaction change by kinetics_delta; U absorbs v (U += v, v = 0) at the
// start and after evaluations at least kRebase steps apart, which keeps v of
// the size of the motion over that many steps (each re-basing costs about one
// FP64 step).  The stop rule compares v with its snapshot taken since, which
// is u^s - u^(s-1).  sm must then hold 2 N (N + 1) doubles.
constexpr int kRebase = 200;

template <typename T, int N, int SPL, bool VF, typename MD, bool LOAD, typename TS, bool RF = false>
__device__ __forceinline__ int fused_q_solve(T *sm, double *red, int *sbad, const DevSolve &s, int b, T *state,
                                             TS *out, const T *tables, double dt, const PersistArgs &pa,
                                             long long &step, T (&ur)[SPL][N / 8], T (&ui)[SPL][N / 8],
                                             double *u64 = nullptr)
{
    static_assert(!RF || std::is_same<T, float>::value, "the refinement form steps its correction in FP32");
    // split-step twiddles in registers where the register budget allows
    // (the refinement form keeps U in registers: w and ph only)
    constexpr int CT = sizeof(T) * N > 256 ? 0 : (RF ? 1 : 2);
    using Q = QuadLine<T, N, CT>;
    constexpr int P = Q::P, M = N / 2;
    constexpr int LD = N + 1, SP = N * LD, NN = N * N;
    constexpr int THREADS = (8 / SPL) * N, WAVES = THREADS / 64;
    const int tid = threadIdx.x;
    const int g = SPL == 2 ? tid >> 2 : tid >> 3;
    const int sp0 = SPL == 2 ? 0 : (tid >> 2) & 1;          // the lane's first species
    const int q = (SPL == 1 && sp0) ? 3 - (tid & 3) : (tid & 3);
    typename Q::Lane L;
    Q::init(L, q);
    const T p[4] = {T(s.p[0]), T(s.p[1]), T(s.p[2]), T(s.p[3])};
    const T tdt = T(dt);
    const int kb = P * L.k2;
    // Addresses: a uniform base, a per-lane offset and a compile-time offset
    // that is never negative (so LDS and buffer instructions take it as an
    // immediate).  Line values: pairs m1 < P/2 at lo + 16 m1 + 2h, the others
    // at hi - 16 m1 - 2h = hi0 + (16 (P - 1) + 2 - 16 m1 - 2h).
    constexpr int HI_SPAN = 16 * (P - 1) + 2;
    const int lo = Q::template pos_base<0>(q), hi0 = Q::template pos_base<P - 1>(q) - HI_SPAN;
    auto line_off = [&](auto m1c, auto hc) {        // offset of a line value from its base
        constexpr int m1 = decltype(m1c)::value, h = decltype(hc)::value;
        return m1 < P / 2 ? 16 * m1 + 2 * h : HI_SPAN - 16 * m1 - 2 * h;
    };
    const auto ub = make_rsrc(state + s.off, 2 * NN * sizeof(T));                    // the solve's state
    const unsigned hu0 = (sp0 * NN + g * N + lo) * sizeof(T), hu1 = (sp0 * NN + g * N + hi0) * sizeof(T);
    T *const smp = sm + sp0 * SP;
    T *const cb0 = smp + lo * LD + g, *const cb1 = smp + hi0 * LD + g;   // column g, first species
    T *const rk = smp + g * LD + kb;                            // X_k of row g at rk[k1]
    T *const rn = smp + g * LD + (N - kb) - (P - 1);            // X_{N-k} at rn[P - 1 - k1]
    T *const rm = smp + g * LD + M;
    // Spectral divisor of the column pass.  VF: in the split step's V form,
    // [species][A | B | Ci][k = 0..M][l] (k_make_vtables); else the plain
    // divisors [species][k][l] (k_make_tables) applied to X_k and X_{N-k}.
    constexpr int VPL = (M + 1) * N, VSP = VF ? 3 * VPL : NN;
    const auto tb = make_rsrc(tables + (size_t)s.tab * 2 * VSP, 2 * VSP * sizeof(T));
    const unsigned tko = (sp0 * VSP + kb * N + g) * sizeof(T), tmo = (sp0 * VSP + M * N + g) * sizeof(T);
    const unsigned tno = (sp0 * VSP + (N - kb - (P - 1)) * N + g) * sizeof(T);

    // ur/ui: the lane's 2P values of each of its species along row g, natural order
    auto hbm_ld = [&](auto m1c, auto hc, int c) -> T {
        constexpr int m1 = decltype(m1c)::value;
        return buf_load<T>(ub, (m1 < P / 2 ? hu0 : hu1) + line_off(m1c, hc) * sizeof(T), c * NN * sizeof(T));
    };
    auto hbm_st = [&](T v, auto m1c, auto hc, int c) {
        constexpr int m1 = decltype(m1c)::value;
        buf_store<T>(v, ub, (m1 < P / 2 ? hu0 : hu1) + line_off(m1c, hc) * sizeof(T), c * NN * sizeof(T));
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    if constexpr (LOAD) {
        static_for<0, P>([&](auto Mi) {
#pragma unroll
            for (int c = 0; c < SPL; ++c) {
                ur[c][Mi] = hbm_ld(Mi, I0{}, c);
                ui[c][Mi] = hbm_ld(Mi, I1{}, c);
            }
        });
    }
    // refinement form: U rounded to T (own species c at (m1, h); o32 the other
    // species at the same points when SPL == 1) in registers, and R rounded to
    // T in the half of the LDS that the FP32 steps leave free (2 N (N + 1)
    // doubles hold the 2 N^2 floats of the transposes and the 2 N^2 of R):
    // lane-major in groups of four m1, so that each lane's reads are 16-byte
    // and a wavefront's are consecutive.
    constexpr int RP = RF ? P : 1;
    static_assert(!RF || P % 4 == 0, "R is stored in groups of four values");
    T u32[SPL][2][RP], o32[2][(RF && SPL == 1) ? P : 1];
    float4 *const rq = RF ? reinterpret_cast<float4 *>(sm + 2 * SP) + tid : nullptr;
    auto rq_at = [&](int c, int h, int j) -> float4 & { return rq[((c * 2 + h) * (P / 4) + j) * THREADS]; };
    const auto u64r = make_rsrc(RF ? u64 + s.off : nullptr, RF ? 2 * NN * sizeof(double) : 0);
    const unsigned du0 = (sp0 * NN + g * N + lo) * sizeof(double), du1 = (sp0 * NN + g * N + hi0) * sizeof(double);
    auto rebase = [&](bool first) __attribute__((always_inline)) {
        if constexpr (RF) {
            double *const sd = reinterpret_cast<double *>(sm);
            __syncthreads();                                   // the LDS's last readers are done
            static_for<0, P>([&](auto Mi) {
                constexpr int m1 = Mi;
                static_for<0, 2>([&](auto Hc) {
                    constexpr int h = Hc;
                    const int pos = (m1 < P / 2 ? lo : hi0) + line_off(Mi, Hc);
                    const unsigned off = (m1 < P / 2 ? du0 : du1) + line_off(Mi, Hc) * sizeof(double);
    #pragma unroll
                    for (int c = 0; c < SPL; ++c) {
                        double U;
                        if constexpr (h == 0) U = (double)ur[c][m1];
                        else U = (double)ui[c][m1];
                        if (!first) U += buf_load<double>(u64r, off, c * NN * sizeof(double));
                        buf_store<double>(U, u64r, off, c * NN * sizeof(double));
                        sd[(sp0 + c) * SP + g * LD + pos] = U;
                        if constexpr (h == 0) ur[c][m1] = T(0);
                        else ui[c][m1] = T(0);
                    }
                });
            });
            __syncthreads();
            T r32[SPL][2][RP];
            const double pd[4] = {s.p[0], s.p[1], s.p[2], s.p[3]};
            const int gu = g > 0 ? g - 1 : 0, gd = g < N - 1 ? g + 1 : N - 1;
            static_for<0, P>([&](auto Mi) {
                constexpr int m1 = Mi;
                static_for<0, 2>([&](auto Hc) {
                    constexpr int h = Hc;
                    const int pos = (m1 < P / 2 ? lo : hi0) + line_off(Mi, Hc);
                    const int pl = pos > 0 ? pos - 1 : 0, pr = pos < N - 1 ? pos + 1 : N - 1;
    #pragma unroll
                    for (int c = 0; c < SPL; ++c) {
                        const int cs = sp0 + c;
                        const double *const fld = sd + cs * SP;
                        const double U0 = fld[g * LD + pos];
                        const double Uo = sd[(1 - cs) * SP + g * LD + pos];
                        const double lap =
                            (fld[g * LD + pl] + fld[g * LD + pr] + fld[gu * LD + pos] + fld[gd * LD + pos] - 4.0 * U0) *
                            s.inv_h2;
                        double f, gg;
                        kinetics<MD::value>(pd, cs ? Uo : U0, cs ? U0 : Uo, f, gg);
                        r32[c][h][m1] = (T)((cs ? gg : f) + (cs ? s.nu[1] : s.nu[0]) * lap);
                        u32[c][h][m1] = (T)U0;
                        if constexpr (SPL == 1) o32[h][m1] = (T)Uo;
                    }
                });
            });
            __syncthreads();                                   // the FP64 field's last readers are done
#pragma unroll
            for (int c = 0; c < SPL; ++c)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int j = 0; j < P / 4; ++j)
                        rq_at(c, h, j) = make_float4(r32[c][h][4 * j], r32[c][h][4 * j + 1], r32[c][h][4 * j + 2],
                                                     r32[c][h][4 * j + 3]);
            // the row forward writes the LDS's first half next, which these
            // stores do not touch; each lane reads back only its own values
        }
    };
    const long long start = step;
    long long last_rebase = step;
    if constexpr (RF) rebase(true);
    int fin = -1;
    while (true) {
        const bool eval_now = step > start && ((step % pa.check == 0) || step == pa.max_steps);
        if (eval_now) {       // stop rule on u^step against the snapshot of u^(step-1)
            double d = 0.0, a = 0.0;
            int bad = 0;
            static_for<0, P>([&](auto Mi) {
#pragma unroll
                for (int c = 0; c < SPL; ++c) {
                    const T o0 = hbm_ld(Mi, I0{}, c), o1 = hbm_ld(Mi, I1{}, c);
                    const double v0 = (double)ur[c][Mi], v1 = (double)ui[c][Mi];
                    const double d0 = fabs(v0 - (double)o0), d1 = fabs(v1 - (double)o1);
                    bad |= !isfinite(v0) || !isfinite(v1);
                    d = fmax(d, fmax(isnan(d0) ? 0.0 : d0, isnan(d1) ? 0.0 : d1));
                    if constexpr (!RF) a = fmax(a, fmax(isnan(v0) ? 0.0 : fabs(v0), isnan(v1) ? 0.0 : fabs(v1)));
                }
            });
            d = wave_max(d);
            a = wave_max(a);
            bad = wave_or(bad);
            if ((tid & 63) == 0) {
                red[tid >> 6] = d;
                red[WAVES + (tid >> 6)] = a;
                sbad[tid >> 6] = bad;
            }
            __syncthreads();
            double dm = 0.0, am = 0.0;
            int anybad = 0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                dm = fmax(dm, red[w]);
                am = fmax(am, red[WAVES + w]);
                anybad |= sbad[w];
            }
            const double r = dm / dt;
            int st = -1;
            if (anybad) st = CIL_SOLVE_NONFINITE;
            else if (pa.tol > 0.0 && r < pa.tol) st = CIL_SOLVE_OK;
            else if (pa.tol > 0.0 && pa.floor_coef > 0.0 && r < pa.floor_coef * am) st = CIL_SOLVE_FP32_FLOOR;
            else if (step == pa.max_steps) st = pa.tol > 0.0 ? CIL_SOLVE_MAXSTEPS : CIL_SOLVE_OK;
            if (tid == 0) {
                pa.resid[b] = anybad ? (double)NAN : r;
                if (st >= 0) pa.status[b] = st;
            }
            fin = st;
            if (st >= 0) break;
            if (pa.prio > 1.0 && pa.tol > 0.0) set_issue_priority(r / pa.tol, pa.prio);
            if constexpr (RF) {
                if (step - last_rebase >= kRebase) {      // uniform over the workgroup
                    rebase(false);
                    last_rebase = step;
                }
            }
        }
        if (step >= pa.max_steps) break;
        const long long next = step + 1;
        if ((next % pa.check == 0) || next == pa.max_steps) {     // snapshot u^step for the next stop rule
            static_for<0, P>([&](auto Mi) {
#pragma unroll
                for (int c = 0; c < SPL; ++c) {
                    hbm_st(ur[c][Mi], Mi, I0{}, c);
                    hbm_st(ui[c][Mi], Mi, I1{}, c);
                }
            });
        }
        // explicit reaction from old values, into bit-reversed order for the forward
        T xr[SPL][P], xi[SPL][P];
        T r32[SPL][2][RP];                                 // refinement form: R, from the LDS
        if constexpr (RF) {
#pragma unroll
            for (int c = 0; c < SPL; ++c)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int j = 0; j < P / 4; ++j) {
                        const float4 v = rq_at(c, h, j);
                        r32[c][h][4 * j] = v.x;
                        r32[c][h][4 * j + 1] = v.y;
                        r32[c][h][4 * j + 2] = v.z;
                        r32[c][h][4 * j + 3] = v.w;
                    }
        }
        static_for<0, P>([&](auto Mi) {
            constexpr int m1 = Mi;
            constexpr int pb = bitrev(m1, Q::LOGP);
            T f, gg;
            if constexpr (RF && SPL == 2) {               // v + dt (R + f(U + v) - f(U))
                kinetics_delta<MD::value>(p, u32[0][0][m1], u32[1][0][m1], ur[0][m1], ur[1][m1], f, gg);
                xr[0][pb] = ur[0][m1] + tdt * (r32[0][0][m1] + f);
                xr[1][pb] = ur[1][m1] + tdt * (r32[1][0][m1] + gg);
                kinetics_delta<MD::value>(p, u32[0][1][m1], u32[1][1][m1], ui[0][m1], ui[1][m1], f, gg);
                xi[0][pb] = ui[0][m1] + tdt * (r32[0][1][m1] + f);
                xi[1][pb] = ui[1][m1] + tdt * (r32[1][1][m1] + gg);
            } else if constexpr (RF) {
                const T pr = dpp_mov<DPP_HALF_MIRROR>(ur[0][m1]), pi = dpp_mov<DPP_HALF_MIRROR>(ui[0][m1]);
                const T a0 = u32[0][0][m1], o0 = o32[0][m1], a1 = u32[0][1][m1], o1 = o32[1][m1];
                kinetics_delta<MD::value>(p, sp0 ? o0 : a0, sp0 ? a0 : o0, sp0 ? pr : ur[0][m1], sp0 ? ur[0][m1] : pr,
                                          f, gg);
                xr[0][pb] = ur[0][m1] + tdt * (r32[0][0][m1] + (sp0 ? gg : f));
                kinetics_delta<MD::value>(p, sp0 ? o1 : a1, sp0 ? a1 : o1, sp0 ? pi : ui[0][m1], sp0 ? ui[0][m1] : pi,
                                          f, gg);
                xi[0][pb] = ui[0][m1] + tdt * (r32[0][1][m1] + (sp0 ? gg : f));
            } else if constexpr (SPL == 2) {
                kinetics<MD::value>(p, ur[0][m1], ur[1][m1], f, gg);
                xr[0][pb] = ur[0][m1] + tdt * f;
                xr[1][pb] = ur[1][m1] + tdt * gg;
                kinetics<MD::value>(p, ui[0][m1], ui[1][m1], f, gg);
                xi[0][pb] = ui[0][m1] + tdt * f;
                xi[1][pb] = ui[1][m1] + tdt * gg;
            } else {
                const T pr = dpp_mov<DPP_HALF_MIRROR>(ur[0][m1]), pi = dpp_mov<DPP_HALF_MIRROR>(ui[0][m1]);
                kinetics<MD::value>(p, sp0 ? pr : ur[0][m1], sp0 ? ur[0][m1] : pr, f, gg);
                xr[0][pb] = ur[0][m1] + tdt * (sp0 ? gg : f);
                kinetics<MD::value>(p, sp0 ? pi : ui[0][m1], sp0 ? ui[0][m1] : pi, f, gg);
                xi[0][pb] = ui[0][m1] + tdt * (sp0 ? gg : f);
            }
        });
        T xa[SPL][P], xb[SPL][P], xm[SPL];
#pragma unroll
        for (int c = 0; c < SPL; ++c) {
            Q::forward_regs(L, xr[c], xi[c], xa[c], xb[c], xm[c]);
            static_for<0, P>([&](auto Ki) {
                constexpr int k1 = Ki;
                rk[c * SP + k1] = xa[c][k1];
                if (k1 != 0 || kb != 0) rn[c * SP + (P - 1 - k1)] = xb[c][k1];
            });
            if (q == 0) rm[c * SP] = xm[c];
        }
        // The column pass's divisor values are loaded ahead of their use
        // (the first species' before the barrier, a second species' before
        // its column reads), so that the table reads' latency overlaps the
        // barrier and the forward transform instead of stalling the divide.
        T da[P], db[P], dc[VF ? P : 1], dm;
        auto load_div = [&](int c) __attribute__((always_inline)) {
            const int cso = c * VSP * sizeof(T);
            static_for<0, P>([&](auto Ki) {
                constexpr int k1 = Ki;
                if constexpr (VF) {
                    da[k1] = buf_load<T>(tb, tko + k1 * N * sizeof(T), cso);
                    db[k1] = buf_load<T>(tb, tko + k1 * N * sizeof(T), cso + VPL * sizeof(T));
                    dc[k1] = buf_load<T>(tb, tko + k1 * N * sizeof(T), cso + 2 * VPL * sizeof(T));
                } else {
                    da[k1] = buf_load<T>(tb, tko + k1 * N * sizeof(T), cso);
                    if constexpr (k1 == 0) db[0] = buf_load<T>(tb, kb == 0 ? tmo : tno + (P - 1) * N * sizeof(T), cso);
                    else db[k1] = buf_load<T>(tb, tno + (P - 1 - k1) * N * sizeof(T), cso);
                }
            });
            dm = buf_load<T>(tb, tmo, cso);
            __builtin_amdgcn_sched_barrier(0);
        };
        load_div(0);
        __syncthreads();
        // column g: forward, divide, inverse
#pragma unroll
        for (int c = 0; c < SPL; ++c) {
            if (c > 0) load_div(c);
            static_for<0, P>([&](auto Mi) {
                constexpr int m1 = Mi;
                constexpr int pb = bitrev(m1, Q::LOGP);
                const T *cc = (m1 < P / 2 ? cb0 : cb1) + c * SP;
                xr[c][pb] = cc[line_off(Mi, I0{}) * LD];
                xi[c][pb] = cc[line_off(Mi, I1{}) * LD];
            });
            if constexpr (VF) {
                Q::forward_v(L, xr[c], xi[c], xa[c], xb[c], xm[c]);       // xa/xb: Re/Im V_k
                static_for<0, P>([&](auto Ki) {
                    constexpr int k1 = Ki;
                    const T re = xa[c][k1], im = xb[c][k1];
                    xa[c][k1] = da[k1] * re + dc[k1] * im;
                    xb[c][k1] = db[k1] * im + dc[k1] * re;
                });
                xm[c] *= dm;
                Q::inverse_v(L, xa[c], xb[c], xm[c], xr[c], xi[c]);
            } else {
                Q::forward_regs(L, xr[c], xi[c], xa[c], xb[c], xm[c]);
                static_for<0, P>([&](auto Ki) {
                    constexpr int k1 = Ki;
                    xa[c][k1] *= da[k1];
                    xb[c][k1] *= db[k1];
                });
                xm[c] *= dm;
                Q::inverse_regs(L, xa[c], xb[c], xm[c], xr[c], xi[c]);
            }
            static_for<0, P>([&](auto Mi) {
                constexpr int m1 = Mi;
                T *cc = (m1 < P / 2 ? cb0 : cb1) + c * SP;
                cc[line_off(Mi, I0{}) * LD] = xr[c][m1];
                cc[line_off(Mi, I1{}) * LD] = xi[c][m1];
            });
        }
        __syncthreads();
        // row g inverse: u^(step+1)
#pragma unroll
        for (int c = 0; c < SPL; ++c) {
            static_for<0, P>([&](auto Ki) {
                constexpr int k1 = Ki;
                xa[c][k1] = rk[c * SP + k1];
                if constexpr (k1 == 0) xb[c][0] = (kb == 0) ? T(0) : rn[c * SP + (P - 1)];
                else xb[c][k1] = rn[c * SP + (P - 1 - k1)];
            });
            xm[c] = rm[c * SP];
            Q::inverse_regs(L, xa[c], xb[c], xm[c], ur[c], ui[c]);
        }
        step = next;
    }
    if constexpr (RF) {                                    // u = U + v
        static_for<0, P>([&](auto Mi) {
            constexpr int m1 = Mi;
            const unsigned b0 = (m1 < P / 2 ? du0 : du1);
#pragma unroll
            for (int c = 0; c < SPL; ++c) {
                const int so = c * NN * sizeof(double);
                ur[c][m1] = T(buf_load<double>(u64r, b0 + line_off(Mi, I0{}) * sizeof(double), so) + (double)ur[c][m1]);
                ui[c][m1] = T(buf_load<double>(u64r, b0 + line_off(Mi, I1{}) * sizeof(double), so) + (double)ui[c][m1]);
            }
        });
    }
    const auto ob = make_rsrc(out + s.off, 2 * NN * sizeof(TS));
    static_for<0, P>([&](auto Mi) {
#pragma unroll
        for (int c = 0; c < SPL; ++c) {
            buf_store<TS>(TS(ur[c][Mi]), ob, (Mi < P / 2 ? hu0 : hu1) / sizeof(T) * sizeof(TS) +
                                                 line_off(Mi, I0{}) * sizeof(TS), c * NN * sizeof(TS));
            buf_store<TS>(TS(ui[c][Mi]), ob, (Mi < P / 2 ? hu0 : hu1) / sizeof(T) * sizeof(TS) +
                                                 line_off(Mi, I1{}) * sizeof(TS), c * NN * sizeof(TS));
        }
    });
    if (tid == 0) pa.steps[b] = step;
    return fin;
}

// Quad variant: every line is transformed by a quad of lanes (dct_quad.hpp);
// each workgroup runs one solve.  Between steps the state is kept in LDS as
// the row-spectral field (after the column inverse).  One step is two passes,
// each ending with the workgroup barrier:
//   row pass     row inverse (u^s in registers), stop rule and snapshot at
//                evaluation steps, explicit reaction (both species of a point
//                in one lane, or in lanes t and t ^ 7), row forward -> LDS;
//   column pass  column forward, spectral divide, column inverse, all in
//                registers (the split-step partners come by DPP) -> LDS.
// The first row pass loads u from HBM instead; the last stores it there.
// One kernel per model (the host picks it), so that each model's step gets a
// register allocation of its own.  WPE is the occupancy the register
// allocation aims at (waves per SIMD).
template <int MODEL, typename T, int N, int SPL, int WPE, bool VF>
__global__ __launch_bounds__((8 / SPL) * N) __attribute__((amdgpu_waves_per_eu(WPE))) void k_fused_q(
    const DevSolve *S, const int *list, T *state, const T *tables, double dt, PersistArgs pa)
{
    constexpr int LD = N + 1, SP = N * LD, WAVES = (8 / SPL) * N / 64;
    __shared__ T sm[2 * SP];
    __shared__ double red[2 * WAVES];
    __shared__ int sbad[WAVES];
    const int b = list[blockIdx.x];
    const DevSolve s = S[b];
    long long step = pa.steps[b];
    T ur[SPL][N / 8], ui[SPL][N / 8];
    fused_q_solve<T, N, SPL, VF, std::integral_constant<int, MODEL>, true, T>(sm, red, sbad, s, b, state, state,
                                                                             tables, dt, pa, step, ur, ui);
}

// FP32 stepping with the polish in one persistent launch.  A solve that
// stops at the FP32 floor continues to the tolerance either with FP64 steps
// (its registers converted, FP64 tables, FP64 snapshots for its stop rule in
// state64) or, with RF, in the refinement form (FP64 state in state64, FP32
// correction steps; tab64 unused); its final state is stored as FP32.
// switch_step[b]: the step at which solve b stopped its FP32 phase.
// mode 0: both phases in this launch; 1: the FP32 phase only (solves at the
// floor keep that status); 2: the second phase only, for solves that a
// mode-1 launch left at their floor (the FP32 phase takes no step: it loads
// the state and stores it back unchanged).  A mode-1 launch followed by a
// mode-2 launch runs the same instructions as one mode-0 launch, so the two
// give the same bits.  One kernel per model, so that each model's two phases
// get a register allocation of their own.
template <int MODEL, int N, int SPL, bool VF32, bool VF64, bool RF>
__global__ __launch_bounds__((8 / SPL) * N) __attribute__((amdgpu_waves_per_eu(2))) void k_fused_q_mixed(
    const DevSolve *S, const int *list, float *state, double *state64, const float *tab32, const double *tab64,
    double dt, PersistArgs pa32, PersistArgs pa64, long long *switch_step, int mode)
{
    constexpr int LD = N + 1, SP = N * LD, WAVES = (8 / SPL) * N / 64, P = N / 8;
    __shared__ __align__(16) double sm[2 * SP];
    __shared__ double red[2 * WAVES];
    __shared__ int sbad[WAVES];
    const int b = list[blockIdx.x];
    const DevSolve s = S[b];
    long long step = pa32.steps[b];
    if (mode == 2) pa32.max_steps = step;
    [&](auto MD) {
        float ur[SPL][P], ui[SPL][P];
        const int fin = fused_q_solve<float, N, SPL, VF32, decltype(MD), true, float>(
            reinterpret_cast<float *>(sm), red, sbad, s, b, state, state, tab32, dt, pa32, step, ur, ui);
        const long long sw = step;
        const bool go = mode == 2 || (mode == 0 && fin == CIL_SOLVE_FP32_FLOOR);   // uniform over the workgroup
        if constexpr (RF) {
            if (go)
                fused_q_solve<float, N, SPL, VF32, decltype(MD), false, float, true>(
                    reinterpret_cast<float *>(sm), red, sbad, s, b, state, state, tab32, dt, pa64, step, ur, ui,
                    state64);
        } else if (go) {
            double vr[SPL][P], vi[SPL][P];
#pragma unroll
            for (int c = 0; c < SPL; ++c)
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    vr[c][m] = (double)ur[c][m];
                    vi[c][m] = (double)ui[c][m];
                }
            __syncthreads();                         // the LDS is reused at double width
            fused_q_solve<double, N, SPL, VF64, decltype(MD), false, float>(sm, red, sbad, s, b, state64, state, tab64,
                                                                            dt, pa64, step, vr, vi);
        }
        if (threadIdx.x == 0 && mode != 2) switch_step[b] = sw;
    }(std::integral_constant<int, MODEL>{});
}

template <typename T, int N, int SPL, int WPE, bool VF>
void launch_q1(int nl, const DevSolve *S, const int *list, T *state, const T *tables, int model, double dt,
               const PersistArgs &pa, hipStream_t st)
{
    dispatch_model(model, [&](auto MD) {
        hipLaunchKernelGGL((k_fused_q<decltype(MD)::value, T, N, SPL, WPE, VF>), dim3(nl), dim3((8 / SPL) * N), 0, st,
                           S, list, state, tables, dt, pa);
    });
}

template <typename T, int N>
void launch_q(int shape, int nl, const DevSolve *S, const int *list, T *state, const T *tables, int model, double dt,
              const PersistArgs &pa, hipStream_t st)
{
    switch (shape) {
    case 0: launch_q1<T, N, 2, 2, false>(nl, S, list, state, tables, model, dt, pa, st); break;
    case 1: launch_q1<T, N, 1, 2, false>(nl, S, list, state, tables, model, dt, pa, st); break;
    case 2: launch_q1<T, N, 2, 2, true>(nl, S, list, state, tables, model, dt, pa, st); break;
    default: launch_q1<T, N, 1, 2, true>(nl, S, list, state, tables, model, dt, pa, st); break;
    }
}

}  // namespace cil
