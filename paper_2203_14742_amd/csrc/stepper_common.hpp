// Device-side pieces shared by the stepper's translation units: the solve
// descriptor, the Sec. 4.1 kinetics, wave reductions and the persistent
// kernels' stop-rule arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "cil.h"
#include "cil_internal.hpp"

namespace cil {

struct DevSolve {
    int64_t off;     // element offset of the solve's state
    int32_t n;
    int32_t tab;     // spectral-table index (fused back-end)
    double inv_h2;   // 1/h^2, h = L/(n-1)
    double nu[2];
    double p[4];
};

struct StepResults {               // indexed by solve
    unsigned long long *resid;     // bits of a non-negative double: max |du|
    unsigned long long *maxabs;    // bits of max |u|
    int *bad;                      // non-finite value seen
};

// 1/w from the hardware reciprocal and Newton steps e = 1 - w r, r += r e
// (two in FP64, one in FP32): within about one unit in the last place of
// the correctly rounded quotient, at half the instructions of IEEE division.
template <typename T>
__device__ __forceinline__ T recip(T w)
{
    if constexpr (sizeof(T) == 8) {
        double r = __builtin_amdgcn_rcp(w);
        double e = fma(-w, r, 1.0);
        r = fma(r, e, r);
        e = fma(-w, r, 1.0);
        return fma(r, e, r);
    } else {
        const float r = __builtin_amdgcn_rcpf(w);
        return fmaf(r, fmaf(-w, r, 1.0f), r);
    }
}

// -------------------------------------------------------------- kinetics
// Sec. 4.1 reaction terms; the model is uniform over a launch.
template <int MODEL, typename T>
__device__ __forceinline__ void kinetics(const T *p, T v, T w, T &f, T &g)
{
    if constexpr (MODEL == CIL_FHN) {
        f = p[1] * (w - p[2] * v);
        g = -v + p[0] * w - w * w * w;
    } else if constexpr (MODEL == CIL_GM) {
        f = -p[0] * v + v * v * recip(w);
        g = -p[1] * w + v * v;
    } else if constexpr (MODEL == CIL_GM_SOURCE) {
        f = p[0] - p[1] * v + v * v * recip(w);
        g = v * v - w;
    } else if constexpr (MODEL == CIL_BRUSSELATOR) {
        f = p[0] - (p[1] + T(1)) * v + v * v * w;
        g = p[1] * v - v * v * w;
    } else {
        f = T(0);
        g = T(0);
    }
}

// The change of the Sec. 4.1 reaction terms between the point (v, w) = (a, b)
// and (a + x, b + y): df = f(a + x, b + y) - f(a, b), dg likewise, expanded
// so that only terms of order x or y remain (no difference of O(1) values
// cancels).  Evaluated in T at a rounded (a, b), the error is a few units of
// T relative to the change itself, however small the change.
template <int MODEL, typename T>
__device__ __forceinline__ void kinetics_delta(const T *p, T a, T b, T x, T y, T &df, T &dg)
{
    if constexpr (MODEL == CIL_FHN) {
        df = p[1] * (y - p[2] * x);
        dg = -x + p[0] * y - y * (T(3) * b * (b + y) + y * y);        // (b + y)^3 - b^3
    } else if constexpr (MODEL == CIL_GM || MODEL == CIL_GM_SOURCE) {
        const T sq = (a + a + x) * x;                                   // (a + x)^2 - a^2
        const T dq = (sq * b - a * a * y) * recip(b * (b + y));         // (a + x)^2/(b + y) - a^2/b
        if constexpr (MODEL == CIL_GM) {
            df = -p[0] * x + dq;
            dg = -p[1] * y + sq;
        } else {
            df = -p[1] * x + dq;
            dg = sq - y;
        }
    } else if constexpr (MODEL == CIL_BRUSSELATOR) {
        const T dc = (a + a + x) * x * (b + y) + a * a * y;             // (a + x)^2 (b + y) - a^2 b
        df = -(p[1] + T(1)) * x + dc;
        dg = p[1] * x - dc;
    } else {
        df = T(0);
        dg = T(0);
    }
}

template <typename F>
__host__ __device__ __forceinline__ void dispatch_model(int model, F &&f)
{
    switch (model) {
    case CIL_FHN: f(std::integral_constant<int, CIL_FHN>{}); break;
    case CIL_GM: f(std::integral_constant<int, CIL_GM>{}); break;
    case CIL_GM_SOURCE: f(std::integral_constant<int, CIL_GM_SOURCE>{}); break;
    case CIL_BRUSSELATOR: f(std::integral_constant<int, CIL_BRUSSELATOR>{}); break;
    default: f(std::integral_constant<int, CIL_HEAT>{}); break;
    }
}

__device__ __forceinline__ inline double wave_max(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ __forceinline__ inline int wave_or(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
    return x;
}

struct PersistArgs {
    long long max_steps;
    double tol;
    int check;
    double floor_coef;          // FP32 stepping: floor_ulps 2^-24 / dt, so the floor is floor_coef max|u|; 0 = off
    long long *steps;           // per solve: steps taken (in: start, out: end)
    double *resid;              // per solve: residual of the last evaluated step
    int *status;                // per solve: cil_solve_status
    double prio;                // > 1: issue priority by distance from tol in powers of prio; 0: off
};

// A residual-stopped batch ends with its slowest solve.  With `prio`, a solve
// far from its tolerance (many steps to go) takes issue priority on its SIMDs
// over a co-resident solve that is nearly done (s_setprio, wave level).
__device__ __forceinline__ void set_issue_priority(double ratio, double base)
{
    if (ratio > base * base * base) __builtin_amdgcn_s_setprio(3);
    else if (ratio > base * base) __builtin_amdgcn_s_setprio(2);
    else if (ratio > base) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// Mixed-precision quad launch (stepper_quad_mixed.hip): n = 32 and 64 with the
// default shapes (FP32 shape 1 / FP64 shape 1 at n = 32, 2 / 0 at n = 64).
// refine = 1: the continuation is the refinement form (FP64 state in state64,
// FP32 correction steps; tab64 unused), else FP64 steps.  mode 0: both
// phases; 1: the FP32 phase only; 2: the continuation only (k_fused_q_mixed).
int launch_quad_mixed(int n, int nl, const DevSolve *S, const int *list, float *state, double *state64,
                      const float *tab32, const double *tab64, int model, double dt, const PersistArgs &pa32,
                      const PersistArgs &pa64, long long *switch_step, int refine, int mode, hipStream_t st);

// Quad-variant launch, one translation unit per precision (stepper_quad_*.hip).
int launch_quad_f32(int n, int shape, int nl, const DevSolve *S, const int *list, float *state, const float *tables,
                    int model, double dt, const PersistArgs &pa, hipStream_t st);
int launch_quad_f64(int n, int shape, int nl, const DevSolve *S, const int *list, double *state, const double *tables,
                    int model, double dt, const PersistArgs &pa, hipStream_t st);

// Code shapes of the quad variant: species per lane, the occupancy the
// register allocation aims at, and the form of the column-pass divisor (V
// form: fewer operations, one more table plane).  Chosen per (precision, n)
// from measurements; cil_set_option(CIL_OPT_QUAD_SHAPE) overrides.
struct QuadShape {
    int spl, wpe, vform;
};
constexpr int kQuadShapes = 4;
constexpr QuadShape kQuadShape[kQuadShapes] = {{2, 2, 0}, {1, 2, 0}, {2, 2, 1}, {1, 2, 1}};

}  // namespace cil
