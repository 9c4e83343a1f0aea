// Internal declarations shared by the HIP translation units of libcil.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>
#include <utility>

#include "../../include/cil.h"

namespace cil {

// ------------------------------------------------------------------ errors
int set_error(int code, const char *fmt, ...);
void clear_error();

#define CIL_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return ::cil::set_error(CIL_EDEVICE, "%s failed: %s (%s:%d)", #expr,         \
                                    hipGetErrorString(_e), __FILE__, __LINE__);         \
    } while (0)

#define CIL_TRY(expr)                                                                   \
    do {                                                                                \
        int _rc = (expr);                                                               \
        if (_rc != CIL_OK) return _rc;                                                  \
    } while (0)

// -------------------------------------------------------------- workspaces
// Grow-only device buffers, one per (device, slot).  Contents are not kept
// across calls unless the caller says so.  Freed by cil_shutdown().
enum WsSlot {
    WS_STEP_SOLVES = 0, WS_STEP_LIST, WS_STEP_RESID, WS_STEP_TABLES, WS_STEP_WORK_A,
    WS_STEP_WORK_B, WS_STEP_STATE64, WS_STEP_LIST64, WS_STEP_DCT,
    WS_DIST_NORMS, WS_DIST_SPLIT_A, WS_DIST_SPLIT_B, WS_DIST_RECHECK, WS_DIST_COUNTS,
    WS_DIST_MISC, WS_DIST_SAMPLE, WS_BOOT_MISC, WS_BOOT_MULT, WS_STATS_MISC, WS_FEAT_MISC, WS_FEAT_SEG,
    WS_DIST_REDUCED,
    WS_NUM_SLOTS
};
int ws_get(int slot, size_t bytes, void **ptr);
// Pinned host buffers for the small copies between the host and the device
// inside a call (so they run asynchronously), grow-only, one per (device,
// slot); freed by cil_shutdown().
enum HostSlot { HS_DIST = 0, HS_BOOT, HS_STEP, HS_NUM_SLOTS };
int host_stage(int slot, size_t bytes, void **ptr);
int current_device(int *dev);
// Wait for everything issued to `st` (polls, then blocks; CIL_OPT_SYNC_SPIN_US).
int stream_wait(hipStream_t st);
int release_all();
// Zero device memory with a kernel (keeps memset nodes out of captured graphs).
int fill_zero(void *p, size_t bytes, hipStream_t st);

// ---------------------------------------------------------------- profiler
// When enabled (cil_profile), hot kernel launches are bracketed by HIP events
// recorded on the launch stream; durations are accumulated per kernel name.
bool prof_enabled();
struct ProfMark {
    int slot = -1;
};
ProfMark prof_begin(const char *name, hipStream_t st);
void prof_end(ProfMark m, hipStream_t st);
void prof_flush();

// --------------------------------------------------------- launch checks
inline int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(CIL_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
    return CIL_OK;
}

// ------------------------------------------------- compile-time cos / sin
// cos(pi p / q) and sin(pi p / q) for integers p, q > 0, evaluated at
// compile time: exact octant reduction in integers, then a Taylor series on
// [0, pi/4].  Accurate to about one ulp in double; used for FFT twiddles,
// which then become instruction literals.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ce_sin_series(double x)
{
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k < 15; ++k) {
        term *= -x2 / (double)((2 * k) * (2 * k + 1));
        sum += term;
    }
    return sum;
}

constexpr double ce_cos_series(double x)
{
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 15; ++k) {
        term *= -x2 / (double)((2 * k - 1) * (2 * k));
        sum += term;
    }
    return sum;
}

constexpr double ce_cospi(long p, long q)
{
    long r = p % (2 * q);
    if (r < 0) r += 2 * q;          // [0, 2q)
    if (r > q) r = 2 * q - r;       // cos is even about pi: [0, q]
    double sign = 1.0;
    if (2 * r > q) {                // (pi/2, pi]: cos(t) = -cos(pi - t)
        r = q - r;
        sign = -1.0;
    }
    if (4 * r > q)                  // (pi/4, pi/2]: cos(t) = sin(pi/2 - t)
        return sign * ce_sin_series(kPi * (double)(q - 2 * r) / (double)(2 * q));
    return sign * ce_cos_series(kPi * (double)r / (double)q);
}

constexpr double ce_sinpi(long p, long q) { return ce_cospi(q - 2 * p, 2 * q); }

// Pattern features beyond L2 (features.hip).
int minmax_scale_impl(const void *X, long long count, int n, cil_precision prec, void *Y, hipStream_t st);
int augment_impl(const void *X, long long count, int n, double L, cil_precision prec, void *Y, hipStream_t st);
int pair_maxabs_impl(const void *A, long long nA, const void *B, long long nB, long long dim, cil_precision prec,
                     const int64_t *seg_end, int nseg, double *D, hipStream_t st);
int combine_segments_impl(const double *D, long long n, int nseg, int mode, double *out, hipStream_t st);
int value_range_impl(const double *V, long long n, double *vmin, double *vmax, hipStream_t st);
int bin_values_impl(const double *V, long long n, const double *radii, int M, uint8_t *bins, int64_t *counts,
                    hipStream_t st);

// Gram FP32 -> FP64 promotion interval (gram.hip), shared with the error bound.
int gram_flush_interval();
int set_gram_flush_interval(int64_t v);
int set_gram_pipeline(int64_t v);
int set_wave_priority(int64_t v);
int set_polish_separate(int64_t v);

// Simulate plans (stepper.hip): a batch of fused solves bound to one graph.
struct SimPlan;
int plan_create(cil_model model, cil_precision prec, const cil_problem *probs, int B, void *state, const int64_t *offs,
                const cil_stepping *stp, hipStream_t st, SimPlan **out);
int plan_tune(SimPlan *p, int64_t steps, hipStream_t st);
int plan_launch(SimPlan *p, hipStream_t st);
int plan_report(SimPlan *p, cil_solve_report *reports, hipStream_t st);
int plan_groups(const SimPlan *p);
int plan_group_info(const SimPlan *p, int g, int *n, int *count, int *shape, double *tuned_ms);
void plan_destroy(SimPlan *p);

// Radii ladder from a squared-distance range (host; shared by cil_radii and the
// adaptive counting call so both give the same doubles).
int radii_ladder(double d2min, double d2max, int M, int law, double *radii);

// ------------------------------------------------------- buffer accesses
// Raw buffer loads/stores: the base lives in a uniform resource (SGPRs), so a
// lane address is one 32-bit byte offset plus compile-time offsets, instead
// of a 64-bit VGPR pair per distinct address.  Accesses past `bytes` read 0
// and are dropped on store.  Resource word 3 = 0x00020000 (gfx9 family).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, unsigned voff, int soff)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                              voff, soff, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

// ------------------------------------------------------------ static_for
template <int I, int N, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int x, int bits)
{
    int r = 0;
    for (int i = 0; i < bits; ++i)
        if (x & (1 << i)) r |= 1 << (bits - 1 - i);
    return r;
}

}  // namespace cil
