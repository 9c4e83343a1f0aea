// extern "C" entry points of libcil: argument validation, device checks,
// workspaces and dispatch to the kernels.  See include/cil.h for the
// contract of every function.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cil_internal.hpp"
#include "distance_async.hpp"

namespace cil {

// implemented in the other translation units
int simulate_impl(cil_model, cil_precision, const cil_problem *, int, void *, const int64_t *,
                  const cil_stepping *, cil_solve_report *, hipStream_t, int scheme);
template <typename T>
int pair_bins_impl(const T *, long long, const T *, long long, long long, const double *, int, uint8_t *,
                   std::vector<unsigned long long> &, hipStream_t);
template <typename T>
int adaptive_bins_impl(const T *, long long, const T *, long long, long long, int, int, int, double *, double *,
                       double *, uint8_t *, std::vector<unsigned long long> &, hipStream_t);
template <typename T>
int distance_range_impl(const T *, long long, const T *, long long, long long, int, double *, double *,
                        hipStream_t);
template <typename T>
int canonical_pairs_impl(const T *, long long, const T *, long long, long long, const long long *,
                         const long long *, long long, double *, hipStream_t);
template <typename T>
int approx_d2_impl(const T *, long long, const T *, long long, long long, double *, double *, hipStream_t);
int bootstrap_impl(const uint8_t *, long long, long long, int, const int *, int, const int *, int, int,
                   long long *, double *, hipStream_t);
int bootstrap_noalloc_impl(const uint8_t *, long long, long long, int, const int *, int, const int *, int, int,
                   long long *, double *, hipStream_t);
int loglik_impl(const double *, int, int, int, const double *, double *, double *, int *, int *,
                hipStream_t);
template <typename T>
int adaptive_bins_async(const T *, long long, const T *, long long, long long, int, int, int, double *, double *,
                        double *, uint8_t *, AsyncBins *, hipStream_t);
int bootstrap_deferred(const uint8_t *, long long, long long, int, const int *, int, const int *, int, int, double *,
                       hipStream_t, int **);
int observed_from_hist(const unsigned long long *, int, double, double *, hipStream_t);
void set_distance_stats(long long, long long, long long);
int range_init_stage(unsigned long long **);
int last_distance_stats(int64_t *, int64_t *, int64_t *);
void set_force_exact(int);
int set_quad_shape(int64_t);
int stepper_release();
void set_boot_gather(int);

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string t_err;
}

int set_error(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

void clear_error() { t_err.clear(); }

// -------------------------------------------------------------- workspaces
namespace {
std::mutex g_ws_mu;
struct WsEntry {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::map<std::pair<int, int>, WsEntry> g_ws;
std::map<int, bool> g_dev_ok;
}  // namespace

int current_device(int *dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return set_error(CIL_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    return CIL_OK;
}

static int check_device()
{
    int dev;
    CIL_TRY(current_device(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_dev_ok.find(dev);
    if (it != g_dev_ok.end()) return it->second ? CIL_OK : set_error(CIL_EDEVICE, "device %d is not gfx950", dev);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return set_error(CIL_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    const bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    g_dev_ok[dev] = ok;
    if (!ok) return set_error(CIL_EDEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    return CIL_OK;
}

int ws_get(int slot, size_t bytes, void **ptr)
{
    int dev;
    CIL_TRY(current_device(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    WsEntry &w = g_ws[std::make_pair(dev, slot)];
    if (w.bytes < bytes) {
        if (w.ptr) (void)hipFree(w.ptr);
        w.ptr = nullptr;
        w.bytes = 0;
        size_t want = bytes + bytes / 4 + 256;
        if (hipMalloc(&w.ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            w.ptr = nullptr;
            return set_error(CIL_ENOMEM, "workspace allocation of %zu bytes failed", want);
        }
        w.bytes = want;
    }
    *ptr = w.ptr;
    return CIL_OK;
}

namespace {
std::map<std::pair<int, int>, WsEntry> g_hs;
}  // namespace

int host_stage(int slot, size_t bytes, void **ptr)
{
    int dev;
    CIL_TRY(current_device(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    WsEntry &w = g_hs[std::make_pair(dev, slot)];
    if (w.bytes < bytes) {
        if (w.ptr) (void)hipHostFree(w.ptr);
        w.ptr = nullptr;
        w.bytes = 0;
        const size_t want = std::max<size_t>(bytes, 64 * 1024);
        if (hipHostMalloc(&w.ptr, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            w.ptr = nullptr;
            return set_error(CIL_ENOMEM, "pinned host buffer of %zu bytes failed", want);
        }
        w.bytes = want;
    }
    *ptr = w.ptr;
    return CIL_OK;
}

// Host waits.  A blocking wait puts the host thread to sleep until the
// device signals; the statistic's short launches are waited on for tens of
// microseconds at a time, about what the wake-up costs.  So the stream's work
// is recorded as an event and polled first, for up to g_spin_us microseconds
// (CIL_OPT_SYNC_SPIN_US), then waited on blocking.  One event per (thread,
// device), kept for the thread's life.
std::atomic<long long> g_spin_us{200000};

int set_sync_spin(int64_t us)
{
    if (us < 0 || us > 10000000) return set_error(CIL_EINVAL, "sync spin %lld us out of range [0, 1e7]", (long long)us);
    g_spin_us.store(us);
    return CIL_OK;
}

int stream_wait(hipStream_t st)
{
    const long long budget = g_spin_us.load();
    if (budget <= 0) {
        CIL_HIP(hipStreamSynchronize(st));
        return CIL_OK;
    }
    int dev;
    CIL_TRY(current_device(&dev));
    thread_local std::map<int, hipEvent_t> evs;
    hipEvent_t &ev = evs[dev];
    if (!ev) CIL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    CIL_HIP(hipEventRecord(ev, st));
    const auto t0 = std::chrono::steady_clock::now();
    while (true) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) return CIL_OK;
        if (e != hipErrorNotReady)
            return set_error(CIL_EDEVICE, "hipEventQuery failed: %s", hipGetErrorString(e));
        const long long us =
            std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now() - t0).count();
        if (us >= budget) break;
    }
    CIL_HIP(hipEventSynchronize(ev));
    return CIL_OK;
}

int release_all()
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_ws) {
        if (kv.second.ptr) {
            (void)hipSetDevice(kv.first.first);
            (void)hipFree(kv.second.ptr);
        }
    }
    for (auto &kv : g_hs)
        if (kv.second.ptr) (void)hipHostFree(kv.second.ptr);
    (void)hipSetDevice(cur);
    g_ws.clear();
    g_hs.clear();
    return CIL_OK;
}

// ---------------------------------------------------------------- profiler
namespace {
std::mutex g_prof_mu;
bool g_prof_on = false;
bool g_prof_steppers_only = false;     // cil_profile(2): the fused stepper kernels only
struct PendingEv {
    std::string name;
    hipEvent_t a, b;
};
std::vector<PendingEv> g_pending;
std::vector<hipEvent_t> g_ev_pool;
struct ProfAcc {
    long long count = 0;
    double total_ms = 0.0;
};
std::map<std::string, ProfAcc> g_prof;

hipEvent_t take_event()
{
    if (!g_ev_pool.empty()) {
        hipEvent_t e = g_ev_pool.back();
        g_ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}
}  // namespace

bool prof_enabled() { return g_prof_on; }

ProfMark prof_begin(const char *name, hipStream_t st)
{
    ProfMark m;
    if (!g_prof_on) return m;
    if (g_prof_steppers_only && strncmp(name, "k_fused", 7) != 0) return m;
    // a stream being captured into a graph gets no timing events
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return m;
    }
    if (cs != hipStreamCaptureStatusNone) return m;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) return m;
    if (hipEventRecord(a, st) != hipSuccess) {
        (void)hipGetLastError();
        return m;
    }
    g_pending.push_back(PendingEv{name, a, b});
    m.slot = (int)g_pending.size() - 1;
    return m;
}

void prof_end(ProfMark m, hipStream_t st)
{
    if (m.slot < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (m.slot < (int)g_pending.size()) (void)hipEventRecord(g_pending[m.slot].b, st);
}

void prof_flush()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &p : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ProfAcc &acc = g_prof[p.name];
            acc.count += 1;
            acc.total_ms += ms;
        } else {
            (void)hipGetLastError();
        }
        g_ev_pool.push_back(p.a);
        g_ev_pool.push_back(p.b);
    }
    g_pending.clear();
}

__global__ void k_fill_zero(unsigned char *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n8 = n / 8;
    if (i < n8) ((unsigned long long *)p)[i] = 0ull;
    if (i < n - 8 * n8) p[8 * n8 + i] = 0;
}

// Zero device memory with a kernel (no memset nodes, so callers may capture).
int fill_zero(void *p, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return CIL_OK;
    if (((uintptr_t)p & 7) != 0) return set_error(CIL_EINVAL, "fill_zero: unaligned pointer");
    const size_t n8 = bytes / 8 + 8;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, st, (unsigned char *)p, bytes);
    return check_launch("k_fill_zero");
}

int radii_ladder(double d2min, double d2max, int M, int law, double *radii)
{
    if (!radii || M < 1) return set_error(CIL_EINVAL, "bad arguments");
    const double R0 = std::sqrt(d2max), RM = std::sqrt(d2min);
    if (!(RM > 0.0) || !(R0 > RM) || !std::isfinite(R0))
        return set_error(CIL_EINVAL, "degenerate distance range [%g, %g]", d2min, d2max);
    if (law == 0) {
        const double b = std::pow(R0 / RM, 1.0 / M);
        for (int m = 1; m <= M; ++m) radii[m - 1] = R0 * std::pow(b, (double)-m);
    } else if (law == 1) {
        const double h = (R0 - RM) / M;
        for (int m = 1; m <= M; ++m) radii[m - 1] = R0 - m * h;
    } else {
        return set_error(CIL_EINVAL, "unknown radius law %d", law);
    }
    return CIL_OK;
}

}  // namespace cil

using namespace cil;

#define API_BEGIN() clear_error()

static bool radii_ok(const double *radii, int M, int maxM)
{
    if (!radii || M < 1 || M > maxM) return false;
    for (int m = 0; m < M; ++m) {
        if (!(radii[m] > 0.0) || !std::isfinite(radii[m])) return false;
        if (m > 0 && !(radii[m] < radii[m - 1])) return false;
    }
    return true;
}

extern "C" {

const char *cil_strerror(int status)
{
    switch (status) {
    case CIL_OK: return "success";
    case CIL_EINVAL: return "invalid argument";
    case CIL_EUNSUPPORTED: return "unsupported";
    case CIL_ENOMEM: return "out of device memory";
    case CIL_EDEVICE: return "device error";
    case CIL_ENOTSPD: return "covariance not positive definite";
    case CIL_ENONFINITE: return "non-finite value";
    default: return "unknown status";
    }
}

const char *cil_last_error(void) { return cil::t_err.c_str(); }

int cil_homogeneous_state(cil_model model, const double *p, double *v0w0)
{
    API_BEGIN();
    if (!p || !v0w0) return set_error(CIL_EINVAL, "null pointer");
    switch (model) {
    case CIL_FHN:
    case CIL_HEAT: v0w0[0] = 0.0; v0w0[1] = 0.0; return CIL_OK;
    case CIL_GM:
        if (!(p[0] != 0.0)) return set_error(CIL_EINVAL, "mu_v must be non-zero");
        v0w0[0] = p[1] / p[0];
        v0w0[1] = p[1] / (p[0] * p[0]);
        return CIL_OK;
    case CIL_GM_SOURCE:
        if (!(p[1] != 0.0)) return set_error(CIL_EINVAL, "b must be non-zero");
        v0w0[0] = (p[0] + 1.0) / p[1];
        v0w0[1] = v0w0[0] * v0w0[0];
        return CIL_OK;
    case CIL_BRUSSELATOR:
        if (!(p[0] != 0.0)) return set_error(CIL_EINVAL, "A must be non-zero");
        v0w0[0] = p[0];
        v0w0[1] = p[1] / p[0];
        return CIL_OK;
    default: return set_error(CIL_EINVAL, "unknown model %d", (int)model);
    }
}

static int simulate_checked(cil_model model, cil_precision prec, const cil_problem *probs, int32_t B, void *state,
                            const int64_t *elem_offsets, const cil_stepping *stepping, cil_solve_report *reports,
                            void *hip_stream, int scheme)
{
    if ((int)model < CIL_FHN || (int)model > CIL_HEAT) return set_error(CIL_EINVAL, "unknown model %d", (int)model);
    if (prec != CIL_FP32 && prec != CIL_FP64) return set_error(CIL_EINVAL, "unknown precision");
    if (B < 0) return set_error(CIL_EINVAL, "B < 0");
    if (B == 0) return CIL_OK;
    if (!probs || !state || !stepping) return set_error(CIL_EINVAL, "null pointer");
    if (!(stepping->dt > 0.0) || !std::isfinite(stepping->dt)) return set_error(CIL_EINVAL, "dt must be > 0");
    if (stepping->max_steps < 0) return set_error(CIL_EINVAL, "max_steps < 0");
    if (stepping->check_every < 1) return set_error(CIL_EINVAL, "check_every < 1");
    if (stepping->path < CIL_PATH_AUTO || stepping->path > CIL_PATH_FUSED_QUAD)
        return set_error(CIL_EINVAL, "unknown path");
    if (stepping->polish < 0 || stepping->polish > 2) return set_error(CIL_EINVAL, "polish must be 0, 1 or 2");
    for (int b = 0; b < B; ++b) {
        const cil_problem &p = probs[b];
        if (p.n < 2 || p.n > 4096) return set_error(CIL_EINVAL, "solve %d: n = %d out of range [2, 4096]", b, p.n);
        if (!(p.L > 0.0) || !std::isfinite(p.L)) return set_error(CIL_EINVAL, "solve %d: L must be > 0", b);
        if (!(p.nu[0] >= 0.0) || !(p.nu[1] >= 0.0)) return set_error(CIL_EINVAL, "solve %d: nu must be >= 0", b);
        if (elem_offsets && elem_offsets[b] < 0) return set_error(CIL_EINVAL, "solve %d: negative offset", b);
    }
    CIL_TRY(check_device());
    if (stepping->max_steps == 0) {
        if (reports)
            for (int b = 0; b < B; ++b) reports[b] = cil_solve_report{0, 0, 0.0, CIL_SOLVE_OK, 0};
        return CIL_OK;
    }
    return simulate_impl(model, prec, probs, B, state, elem_offsets, stepping, reports, (hipStream_t)hip_stream,
                         scheme);
}

int cil_simulate_patterns(cil_model model, cil_precision prec, const cil_problem *probs, int32_t B, void *state,
                          const int64_t *elem_offsets, const cil_stepping *stepping, cil_solve_report *reports,
                          void *hip_stream)
{
    API_BEGIN();
    return simulate_checked(model, prec, probs, B, state, elem_offsets, stepping, reports, hip_stream, 0);
}

int cil_simulate_patterns_sbdf2(cil_model model, cil_precision prec, const cil_problem *probs, int32_t B,
                                void *state, const int64_t *elem_offsets, const cil_stepping *stepping,
                                cil_solve_report *reports, void *hip_stream)
{
    API_BEGIN();
    return simulate_checked(model, prec, probs, B, state, elem_offsets, stepping, reports, hip_stream, 1);
}

// plan handles are cil::SimPlan objects behind the opaque C type
static cil::SimPlan *as_plan(cil_sim_plan *p) { return reinterpret_cast<cil::SimPlan *>(p); }
static const cil::SimPlan *as_cplan(const cil_sim_plan *p) { return reinterpret_cast<const cil::SimPlan *>(p); }

int cil_sim_plan_create(cil_model model, cil_precision prec, const cil_problem *probs, int32_t B, void *state,
                        const int64_t *elem_offsets, const cil_stepping *stepping, void *hip_stream,
                        cil_sim_plan **plan)
{
    API_BEGIN();
    if (!plan) return set_error(CIL_EINVAL, "null plan pointer");
    *plan = nullptr;
    if ((int)model < CIL_FHN || (int)model > CIL_HEAT) return set_error(CIL_EINVAL, "unknown model %d", (int)model);
    if (prec != CIL_FP32 && prec != CIL_FP64) return set_error(CIL_EINVAL, "unknown precision");
    if (B < 1) return set_error(CIL_EINVAL, "a plan needs B >= 1");
    if (!probs || !state || !stepping) return set_error(CIL_EINVAL, "null pointer");
    if (!(stepping->dt > 0.0) || !std::isfinite(stepping->dt)) return set_error(CIL_EINVAL, "dt must be > 0");
    if (stepping->max_steps < 0) return set_error(CIL_EINVAL, "max_steps < 0");
    if (stepping->check_every < 1) return set_error(CIL_EINVAL, "check_every < 1");
    if (stepping->path < CIL_PATH_AUTO || stepping->path > CIL_PATH_FUSED_QUAD)
        return set_error(CIL_EINVAL, "unknown path");
    if (stepping->polish < 0 || stepping->polish > 2) return set_error(CIL_EINVAL, "polish must be 0, 1 or 2");
    for (int b = 0; b < B; ++b) {
        const cil_problem &p = probs[b];
        if (p.n < 2 || p.n > 4096) return set_error(CIL_EINVAL, "solve %d: n = %d out of range [2, 4096]", b, p.n);
        if (!(p.L > 0.0) || !std::isfinite(p.L)) return set_error(CIL_EINVAL, "solve %d: L must be > 0", b);
        if (!(p.nu[0] >= 0.0) || !(p.nu[1] >= 0.0)) return set_error(CIL_EINVAL, "solve %d: nu must be >= 0", b);
        if (elem_offsets && elem_offsets[b] < 0) return set_error(CIL_EINVAL, "solve %d: negative offset", b);
    }
    CIL_TRY(check_device());
    cil::SimPlan *p = nullptr;
    CIL_TRY(plan_create(model, prec, probs, B, state, elem_offsets, stepping, (hipStream_t)hip_stream, &p));
    *plan = reinterpret_cast<cil_sim_plan *>(p);
    return CIL_OK;
}

int cil_sim_plan_tune(cil_sim_plan *plan, int64_t steps, void *hip_stream)
{
    API_BEGIN();
    if (!plan) return set_error(CIL_EINVAL, "null plan");
    return plan_tune(as_plan(plan), steps, (hipStream_t)hip_stream);
}

int cil_sim_plan_launch(cil_sim_plan *plan, void *hip_stream)
{
    API_BEGIN();
    if (!plan) return set_error(CIL_EINVAL, "null plan");
    return plan_launch(as_plan(plan), (hipStream_t)hip_stream);
}

int cil_sim_plan_report(cil_sim_plan *plan, cil_solve_report *reports, void *hip_stream)
{
    API_BEGIN();
    if (!plan) return set_error(CIL_EINVAL, "null plan");
    return plan_report(as_plan(plan), reports, (hipStream_t)hip_stream);
}

int cil_sim_plan_groups(const cil_sim_plan *plan)
{
    API_BEGIN();
    if (!plan) return set_error(CIL_EINVAL, "null plan");
    return plan_groups(as_cplan(plan));
}

int cil_sim_plan_group_info(const cil_sim_plan *plan, int32_t group, int32_t *n, int32_t *count, int32_t *shape,
                            double *tuned_ms)
{
    API_BEGIN();
    if (!plan) return set_error(CIL_EINVAL, "null plan");
    return plan_group_info(as_cplan(plan), group, n, count, shape, tuned_ms);
}

int cil_sim_plan_destroy(cil_sim_plan *plan)
{
    API_BEGIN();
    plan_destroy(as_plan(plan));
    return CIL_OK;
}

static int check_sets(const void *A, int64_t nA, const void *B, int64_t nB, int64_t dim, cil_precision prec)
{
    if (prec != CIL_FP32 && prec != CIL_FP64) return set_error(CIL_EINVAL, "unknown precision");
    if (nA < 0 || nB < 0 || dim < 0) return set_error(CIL_EINVAL, "negative size");
    if (nA > 0x7fffffffLL || nB > 0x7fffffffLL) return set_error(CIL_EINVAL, "set too large");
    if ((nA > 0 && !A) || (nB > 0 && !B)) return set_error(CIL_EINVAL, "null set pointer");
    return CIL_OK;
}

int cil_pair_bins(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim, cil_precision prec,
                  const double *radii, int32_t M, uint8_t *bins, int64_t *counts, void *hip_stream)
{
    API_BEGIN();
    CIL_TRY(check_sets(setA, nA, setB, nB, dim, prec));
    if (!radii_ok(radii, M, 255)) return set_error(CIL_EINVAL, "radii must be > 0, finite, strictly decreasing, 1 <= M <= 255");
    CIL_TRY(check_device());
    std::vector<unsigned long long> hist;
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == CIL_FP64)
        CIL_TRY(pair_bins_impl<double>((const double *)setA, nA, (const double *)setB, nB, dim, radii, M, bins, hist, st));
    else
        CIL_TRY(pair_bins_impl<float>((const float *)setA, nA, (const float *)setB, nB, dim, radii, M, bins, hist, st));
    if (counts) {
        unsigned long long run = 0;
        for (int m = M; m >= 1; --m) {       // counts[m-1] = #{bin >= m}
            run += hist[m];
            counts[m - 1] = (int64_t)run;
        }
    }
    return CIL_OK;
}

int cil_features(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim, cil_precision prec,
                 const double *radii, int32_t M, int64_t *counts, double *y, void *hip_stream)
{
    API_BEGIN();
    if (!counts) return set_error(CIL_EINVAL, "counts must not be NULL");
    CIL_TRY(cil_pair_bins(setA, nA, setB, nB, dim, prec, radii, M, nullptr, counts, hip_stream));
    if (y) {
        const double np = (double)nA * (double)nB;
        for (int m = 0; m < M; ++m) y[m] = np > 0 ? (double)counts[m] / np : 0.0;
    }
    return CIL_OK;
}

int cil_distance_range(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim, cil_precision prec,
                       int32_t exclude_diagonal, double *d2min, double *d2max, void *hip_stream)
{
    API_BEGIN();
    CIL_TRY(check_sets(setA, nA, setB, nB, dim, prec));
    if (!d2min || !d2max) return set_error(CIL_EINVAL, "null output");
    if (exclude_diagonal && nA != nB) return set_error(CIL_EINVAL, "exclude_diagonal needs nA == nB");
    const long long np = nA * nB - (exclude_diagonal ? nA : 0);
    if (np <= 0) return set_error(CIL_EINVAL, "no pairs");
    CIL_TRY(check_device());
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == CIL_FP64)
        return distance_range_impl<double>((const double *)setA, nA, (const double *)setB, nB, dim,
                                           exclude_diagonal, d2min, d2max, st);
    return distance_range_impl<float>((const float *)setA, nA, (const float *)setB, nB, dim, exclude_diagonal,
                                      d2min, d2max, st);
}

int cil_canonical_d2(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim, cil_precision prec,
                     const int64_t *ia, const int64_t *jb, int64_t npairs, double *d2, void *hip_stream)
{
    API_BEGIN();
    CIL_TRY(check_sets(setA, nA, setB, nB, dim, prec));
    if (npairs < 0) return set_error(CIL_EINVAL, "negative size");
    if (npairs == 0) return CIL_OK;
    if (!setA || !setB || !ia || !jb || !d2) return set_error(CIL_EINVAL, "null pointer");
    CIL_TRY(check_device());
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == CIL_FP64)
        return canonical_pairs_impl<double>((const double *)setA, nA, (const double *)setB, nB, dim,
                                            (const long long *)ia, (const long long *)jb, npairs, d2, st);
    return canonical_pairs_impl<float>((const float *)setA, nA, (const float *)setB, nB, dim, (const long long *)ia,
                                       (const long long *)jb, npairs, d2, st);
}

int cil_approx_d2(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim, cil_precision prec,
                  double *d2, double *eps, void *hip_stream)
{
    API_BEGIN();
    CIL_TRY(check_sets(setA, nA, setB, nB, dim, prec));
    if (nA * nB == 0) return CIL_OK;
    if (!d2 || !eps) return set_error(CIL_EINVAL, "null output");
    CIL_TRY(check_device());
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == CIL_FP64)
        return approx_d2_impl<double>((const double *)setA, nA, (const double *)setB, nB, dim, d2, eps, st);
    return approx_d2_impl<float>((const float *)setA, nA, (const float *)setB, nB, dim, d2, eps, st);
}

int cil_radii(double d2min, double d2max, int32_t M, int32_t law, double *radii)
{
    API_BEGIN();
    return cil::radii_ladder(d2min, d2max, M, law, radii);
}

int cil_pair_bins_adaptive(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                           cil_precision prec, int32_t exclude_diagonal, int32_t M, int32_t law, double *d2min,
                           double *d2max, double *radii, uint8_t *bins, int64_t *counts, void *hip_stream)
{
    API_BEGIN();
    CIL_TRY(check_sets(setA, nA, setB, nB, dim, prec));
    if (!d2min || !d2max || !radii) return set_error(CIL_EINVAL, "null output");
    if (M < 1 || M > 255) return set_error(CIL_EINVAL, "M must be in [1, 255]");
    if (law != 0 && law != 1) return set_error(CIL_EINVAL, "unknown radius law %d", law);
    if (exclude_diagonal && nA != nB) return set_error(CIL_EINVAL, "exclude_diagonal needs nA == nB");
    if (nA * nB - (exclude_diagonal ? nA : 0) <= 0) return set_error(CIL_EINVAL, "no pairs");
    CIL_TRY(check_device());
    std::vector<unsigned long long> hist;
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == CIL_FP64)
        CIL_TRY(adaptive_bins_impl<double>((const double *)setA, nA, (const double *)setB, nB, dim, exclude_diagonal,
                                           M, law, d2min, d2max, radii, bins, hist, st));
    else
        CIL_TRY(adaptive_bins_impl<float>((const float *)setA, nA, (const float *)setB, nB, dim, exclude_diagonal, M,
                                          law, d2min, d2max, radii, bins, hist, st));
    if (counts) {
        unsigned long long run = 0;
        for (int m = M; m >= 1; --m) {
            run += hist[m];
            counts[m - 1] = (int64_t)run;
        }
    }
    return CIL_OK;
}

}  // extern "C"

namespace {
// 1: the statistic's radii formed on the device and checked against the
// host's at the end (default); 0: formed on the host after a read-back of
// the range; 2: as 1 with the check always failing (tests the fallback).
std::atomic<int> g_stat_radii{1};
struct StatArgs {
    const void *A, *B;
    int64_t nA, nB, dim;
    int prec, M, law;
    const int32_t *idxA, *idxB;
    int32_t kA, kB, n_boot;
    uint8_t *bins;
    double *Y, *y_obs, *f, *loglik;
    int32_t *m_eff, *status;
};

// What the host needs after the stream pass: the pinned read-back locations
// (fixed offsets of the HS_DIST staging) and the list capacity.
struct StatPending {
    unsigned long long *hh, *cnt, *hits;
    int *hb;
    RangeOut *ro;               // null: the radii were formed on the host
    long long cap;
    long long nrange, nrange_exact;
};

// The stream work of Alg. 2bst: range, radii, bins, bootstrap, observed
// vector, likelihood, and the copies of what the host checks into pinned
// staging.  With device_radii no host value enters it after the start: the
// host waits once, at the end.
template <typename T>
int statistic_enqueue(const StatArgs &a, int device_radii, double *d2min, double *d2max, double *radii,
                      hipStream_t st, StatPending *pd)
{
    AsyncBins ab;
    CIL_TRY(adaptive_bins_async<T>((const T *)a.A, a.nA, (const T *)a.B, a.nB, a.dim, a.M, a.law, device_radii, d2min,
                                   d2max, radii, a.bins, &ab, st));
    int *bflags = nullptr;
    CIL_TRY(bootstrap_deferred(a.bins, a.nA, a.nB, a.M, a.idxA, a.kA, a.idxB, a.kB, a.n_boot, a.Y, st, &bflags));
    CIL_TRY(observed_from_hist(ab.hist, a.M, (double)a.nA * (double)a.nB, a.y_obs, st));
    CIL_TRY(loglik_impl(a.Y, 1, a.n_boot, a.M, a.y_obs, a.f, a.loglik, a.m_eff, a.status, st));
    // pinned staging past the range counters' initial values (offset 0)
    char *hs;
    CIL_TRY(host_stage(HS_DIST, 8192, (void **)&hs));
    pd->hh = (unsigned long long *)(hs + 2048);
    pd->cnt = (unsigned long long *)(hs + 4096);
    pd->hb = (int *)(hs + 4096 + 16);
    pd->hits = (unsigned long long *)(hs + 4096 + 32);
    pd->ro = ab.ro ? (RangeOut *)(hs + 4096 + 64) : nullptr;
    pd->cap = ab.cap;
    pd->nrange = ab.nrange;
    pd->nrange_exact = ab.nrange_exact;
    CIL_HIP(hipMemcpyAsync(pd->hh, ab.hist, sizeof(unsigned long long) * (a.M + 1), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipMemcpyAsync(pd->cnt, ab.nlist, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    CIL_HIP(hipMemcpyAsync(pd->hb, bflags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    if (ab.ro) {
        CIL_HIP(hipMemcpyAsync(pd->ro, ab.ro, sizeof(RangeOut), hipMemcpyDeviceToHost, st));
        CIL_HIP(hipMemcpyAsync(pd->hits, ab.nlist + 7, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    }
    return CIL_OK;
}

// After the stream has drained: the checks and the host outputs.
// *mismatch: the device's radii differ from the host's at a threshold with
// a pair near it (the outputs are then those of the device's radii: the
// caller redoes the call with the host's).
int statistic_finish(const StatArgs &a, const StatPending &pd, double *d2min, double *d2max, double *radii,
                     int64_t *counts, bool *mismatch)
{
    *mismatch = false;
    long long nrange = pd.nrange, nrange_exact = pd.nrange_exact;
    if (pd.ro) {
        if (pd.ro->status == 2) return set_error(CIL_ENONFINITE, "non-finite distances in range computation");
        if (pd.ro->status == 3) return set_error(CIL_EDEVICE, "range candidate overflow");
        *d2min = pd.ro->d2min;
        *d2max = pd.ro->d2max;
        CIL_TRY(radii_ladder(*d2min, *d2max, a.M, a.law, radii));      // the degenerate range fails here
        // the host's ladder is the call's; the bins stand unless it differs
        // from the device's at a threshold that has a pair within its window
        unsigned long long differ = 0;
        for (int m = 0; m < a.M; ++m)
            if (std::memcmp(&radii[m], &pd.ro->radii[m], sizeof(double)) != 0) differ |= 1ull << m;
        *mismatch = (differ & *pd.hits) != 0 || g_stat_radii.load() == 2;
        if (*mismatch) return CIL_OK;
        nrange = pd.ro->nrange;
        nrange_exact = pd.ro->nrange_exact;
    }
    if ((long long)pd.cnt[0] > pd.cap) return set_error(CIL_EDEVICE, "re-check list overflow");
    if (pd.hb[0] || pd.hb[1]) return set_error(CIL_EINVAL, "bootstrap index out of range");
    if (counts) {
        unsigned long long run = 0;
        for (int m = a.M; m >= 1; --m) {
            run += pd.hh[m];
            counts[m - 1] = (int64_t)run;
        }
    }
    set_distance_stats(a.nA * a.nB, nrange + (long long)pd.cnt[0], nrange_exact + (long long)pd.cnt[1]);
    return CIL_OK;
}

int statistic_enqueue_any(const StatArgs &a, int device_radii, double *d2min, double *d2max, double *radii,
                          hipStream_t st, StatPending *pd)
{
    if (a.prec == CIL_FP64) return statistic_enqueue<double>(a, device_radii, d2min, d2max, radii, st, pd);
    return statistic_enqueue<float>(a, device_radii, d2min, d2max, radii, st, pd);
}

}  // namespace

static int set_stat_radii(int64_t v)
{
    if (v < 0 || v > 2) return set_error(CIL_EINVAL, "statistic radii option must be 0, 1 or 2");
    g_stat_radii.store((int)v);
    return CIL_OK;
}

extern "C" {

int cil_statistic_adaptive(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim,
                           cil_precision prec, int32_t M, int32_t law, const int32_t *idxA, int32_t kA,
                           const int32_t *idxB, int32_t kB, int32_t n_boot, double *d2min, double *d2max,
                           double *radii, int64_t *counts, uint8_t *bins, double *Y, double *y_obs, double *f,
                           double *loglik, int32_t *m_eff, int32_t *status, void *hip_stream)
{
    API_BEGIN();
    CIL_TRY(check_sets(setA, nA, setB, nB, dim, prec));
    if (!d2min || !d2max || !radii) return set_error(CIL_EINVAL, "null output");
    if (M < 1 || M > 64) return set_error(CIL_EINVAL, "M must be in [1, 64]");
    if (law != 0 && law != 1) return set_error(CIL_EINVAL, "unknown radius law %d", law);
    if (nA * nB <= 0) return set_error(CIL_EINVAL, "no pairs");
    if (kA <= 0 || kB <= 0 || n_boot < 2) return set_error(CIL_EINVAL, "need kA, kB >= 1 and n_boot >= 2");
    if (!idxA || !idxB || !bins || !Y || !y_obs || !f || !loglik || !m_eff || !status)
        return set_error(CIL_EINVAL, "null pointer");
    CIL_TRY(check_device());
    hipStream_t st = (hipStream_t)hip_stream;
    StatArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = setA;
    a.B = setB;
    a.nA = nA;
    a.nB = nB;
    a.dim = dim;
    a.prec = (int)prec;
    a.M = M;
    a.law = law;
    a.idxA = idxA;
    a.idxB = idxB;
    a.kA = kA;
    a.kB = kB;
    a.n_boot = n_boot;
    a.bins = bins;
    a.Y = Y;
    a.y_obs = y_obs;
    a.f = f;
    a.loglik = loglik;
    a.m_eff = m_eff;
    a.status = status;
    int dr = g_stat_radii.load() != 0;
    bool mismatch = false;
    for (int pass = 0; pass < 2; ++pass, dr = 0) {             // a second pass, with the host's radii, after a mismatch
        StatPending pd;
        CIL_TRY(statistic_enqueue_any(a, dr, d2min, d2max, radii, st, &pd));
        CIL_TRY(stream_wait(st));
        CIL_TRY(statistic_finish(a, pd, d2min, d2max, radii, counts, &mismatch));
        if (!mismatch) return CIL_OK;
    }
    return set_error(CIL_EDEVICE, "statistic radii check");
}

int cil_last_distance_stats(int64_t *pairs, int64_t *rechecked, int64_t *exact_fallbacks)
{
    return last_distance_stats(pairs, rechecked, exact_fallbacks);
}

int cil_bootstrap_features(const uint8_t *bins, int64_t nA, int64_t nB, int32_t M, const int32_t *idxA, int32_t kA,
                           const int32_t *idxB, int32_t kB, int32_t n_boot, int64_t *Ycount, double *Y,
                           void *hip_stream)
{
    API_BEGIN();
    if (M < 1 || M > 255) return set_error(CIL_EINVAL, "M must be in [1, 255]");
    if (nA <= 0 || nB <= 0 || kA <= 0 || kB <= 0 || n_boot < 0) return set_error(CIL_EINVAL, "bad sizes");
    if (!bins || !idxA || !idxB) return set_error(CIL_EINVAL, "null pointer");
    CIL_TRY(check_device());
    return bootstrap_impl(bins, nA, nB, M, idxA, kA, idxB, kB, n_boot, (long long *)Ycount, Y,
                          (hipStream_t)hip_stream);
}

int cil_bootstrap_features_noalloc(const uint8_t *bins, int64_t nA, int64_t nB, int32_t M, const int32_t *idxA,
                                   int32_t kA, const int32_t *idxB, int32_t kB, int32_t n_boot, int64_t *Ycount,
                                   double *Y, void *hip_stream)
{
    API_BEGIN();
    if (M < 1 || M > 255) return set_error(CIL_EINVAL, "M must be in [1, 255]");
    if (nA <= 0 || nB <= 0 || kA <= 0 || kB <= 0 || n_boot < 0) return set_error(CIL_EINVAL, "bad sizes");
    if (!bins || !idxA || !idxB) return set_error(CIL_EINVAL, "null pointer");
    CIL_TRY(check_device());
    return bootstrap_noalloc_impl(bins, nA, nB, M, idxA, kA, idxB, kB, n_boot, (long long *)Ycount, Y,
                                  (hipStream_t)hip_stream);
}

int cil_gaussian_loglik(const double *Y, int32_t P, int32_t n_boot, int32_t M, const double *y_obs, double *f,
                        double *loglik, int32_t *m_eff, int32_t *status, void *hip_stream)
{
    API_BEGIN();
    if (P < 0 || n_boot < 2 || M < 1 || M > 64) return set_error(CIL_EINVAL, "need P >= 0, n_boot >= 2, 1 <= M <= 64");
    if (P > 0 && (!Y || !y_obs || !f || !loglik || !m_eff || !status)) return set_error(CIL_EINVAL, "null pointer");
    CIL_TRY(check_device());
    return loglik_impl(Y, P, n_boot, M, y_obs, f, loglik, m_eff, status, (hipStream_t)hip_stream);
}

int cil_minmax_scale(const void *patterns, int64_t count, int32_t n, cil_precision prec, void *out, void *hip_stream)
{
    API_BEGIN();
    if (count < 0 || n < 1) return set_error(CIL_EINVAL, "need count >= 0, n >= 1");
    if (prec != CIL_FP32 && prec != CIL_FP64) return set_error(CIL_EINVAL, "unknown precision");
    if (count > 0 && (!patterns || !out)) return set_error(CIL_EINVAL, "null pointer");
    if (count > 65535) return set_error(CIL_EINVAL, "count > 65535");
    CIL_TRY(check_device());
    return minmax_scale_impl(patterns, count, n, prec, out, (hipStream_t)hip_stream);
}

int cil_augment_patterns(const void *patterns, int64_t count, int32_t n, double L, cil_precision prec, void *out,
                         void *hip_stream)
{
    API_BEGIN();
    if (count < 0 || n < 2) return set_error(CIL_EINVAL, "need count >= 0, n >= 2");
    if (!(L > 0.0) || !std::isfinite(L)) return set_error(CIL_EINVAL, "L must be > 0");
    if (prec != CIL_FP32 && prec != CIL_FP64) return set_error(CIL_EINVAL, "unknown precision");
    if (count > 0 && (!patterns || !out)) return set_error(CIL_EINVAL, "null pointer");
    if (count > 65535) return set_error(CIL_EINVAL, "count > 65535");
    CIL_TRY(check_device());
    return augment_impl(patterns, count, n, L, prec, out, (hipStream_t)hip_stream);
}

int cil_pair_maxabs(const void *setA, int64_t nA, const void *setB, int64_t nB, int64_t dim, cil_precision prec,
                    const int64_t *seg_end, int32_t nseg, double *D, void *hip_stream)
{
    API_BEGIN();
    if (nA < 0 || nB < 0 || dim < 0) return set_error(CIL_EINVAL, "negative size");
    if (prec != CIL_FP32 && prec != CIL_FP64) return set_error(CIL_EINVAL, "unknown precision");
    if (!seg_end) return set_error(CIL_EINVAL, "null segment ends");
    if (nA * nB > 0 && (!setA || !setB || !D)) return set_error(CIL_EINVAL, "null pointer");
    if ((nA + 63) / 64 > 65535) return set_error(CIL_EINVAL, "nA too large");
    CIL_TRY(check_device());
    return pair_maxabs_impl(setA, nA, setB, nB, dim, prec, seg_end, nseg, D, (hipStream_t)hip_stream);
}

int cil_combine_segments(const double *D, int64_t n, int32_t nseg, int32_t mode, double *out, void *hip_stream)
{
    API_BEGIN();
    if (n < 0 || nseg < 1 || mode < 0 || mode > 2) return set_error(CIL_EINVAL, "need n >= 0, nseg >= 1, mode 0..2");
    if (n > 0 && (!D || !out)) return set_error(CIL_EINVAL, "null pointer");
    CIL_TRY(check_device());
    return combine_segments_impl(D, n, nseg, mode, out, (hipStream_t)hip_stream);
}

int cil_value_range(const double *V, int64_t n, double *vmin, double *vmax, void *hip_stream)
{
    API_BEGIN();
    if (n < 1 || !V || !vmin || !vmax) return set_error(CIL_EINVAL, "need n >= 1 and non-null pointers");
    CIL_TRY(check_device());
    return value_range_impl(V, n, vmin, vmax, (hipStream_t)hip_stream);
}

int cil_bin_values(const double *V, int64_t n, const double *radii, int32_t M, uint8_t *bins, int64_t *counts,
                   void *hip_stream)
{
    API_BEGIN();
    if (n < 0 || (n > 0 && !V) || !counts) return set_error(CIL_EINVAL, "bad arguments");
    if (!radii_ok(radii, M, 255)) return set_error(CIL_EINVAL, "radii must be > 0, finite, strictly decreasing, M <= 255");
    CIL_TRY(check_device());
    return bin_values_impl(V, n, radii, M, bins, counts, (hipStream_t)hip_stream);
}

int cil_set_option(int32_t option, int64_t value)
{
    API_BEGIN();
    if (option == 1) {
        set_force_exact((int)value);
        return CIL_OK;
    }
    if (option == CIL_OPT_QUAD_SHAPE) return set_quad_shape(value);
    if (option == CIL_OPT_BOOTSTRAP_GATHER) {
        set_boot_gather((int)value);
        return CIL_OK;
    }
    if (option == CIL_OPT_GRAM_FLUSH) return set_gram_flush_interval(value);
    if (option == CIL_OPT_GRAM_PIPELINE) return set_gram_pipeline(value);
    if (option == CIL_OPT_WAVE_PRIORITY) return set_wave_priority(value);
    if (option == CIL_OPT_POLISH_SEPARATE) return set_polish_separate(value);
    if (option == CIL_OPT_SYNC_SPIN_US) return set_sync_spin(value);
    if (option == CIL_OPT_STAT_DEVICE_RADII) return set_stat_radii(value);
    return set_error(CIL_EINVAL, "unknown option %d", option);
}

int cil_profile(int32_t enable)
{
    API_BEGIN();
    if (enable < 0 || enable > 2) return set_error(CIL_EINVAL, "cil_profile takes 0, 1 or 2");
    prof_flush();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = enable != 0;
    g_prof_steppers_only = enable == 2;
    if (enable) g_prof.clear();
    return CIL_OK;
}

int cil_profile_read(const char *name, int64_t *count, double *total_ms)
{
    API_BEGIN();
    if (!name || !count || !total_ms) return set_error(CIL_EINVAL, "null pointer");
    prof_flush();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    auto it = g_prof.find(name);
    *count = it == g_prof.end() ? 0 : it->second.count;
    *total_ms = it == g_prof.end() ? 0.0 : it->second.total_ms;
    return CIL_OK;
}

int cil_profile_names(char *buf, int64_t len)
{
    API_BEGIN();
    if (!buf || len < 1) return set_error(CIL_EINVAL, "bad buffer");
    prof_flush();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::string s;
    for (auto &kv : g_prof) {
        if (!s.empty()) s += ",";
        s += kv.first;
    }
    if ((int64_t)s.size() + 1 > len) return set_error(CIL_EINVAL, "buffer too small (%zu)", s.size() + 1);
    memcpy(buf, s.c_str(), s.size() + 1);
    return CIL_OK;
}

int cil_shutdown(void)
{
    API_BEGIN();
    prof_flush();
    (void)hipDeviceSynchronize();
    CIL_TRY(stepper_release());
    return release_all();
}

}  // extern "C"
