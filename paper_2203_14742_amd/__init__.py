"""Python binding of libcil, the gfx950 implementation of the Correlation
Integral Likelihood hot path (arXiv 2203.14742).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libcil.so`` (built in-tree by ``paper_2203_14742_amd.build``).  Device
buffers are torch tensors on the current HIP device; calls run on torch's
current stream.  The functions carry the names of the C entry points in
``include/cil.h``; see there for the contract of each.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcil.so")

CIL_OK, CIL_EINVAL, CIL_EUNSUPPORTED, CIL_ENOMEM, CIL_EDEVICE, CIL_ENOTSPD, CIL_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
CIL_FHN, CIL_GM, CIL_GM_SOURCE, CIL_BRUSSELATOR, CIL_HEAT = 0, 1, 2, 3, 4
CIL_FP64, CIL_FP32 = 0, 1
CIL_PATH_AUTO, CIL_PATH_PLAIN, CIL_PATH_FUSED, CIL_PATH_FUSED_LINE, CIL_PATH_FUSED_QUAD = 0, 1, 2, 3, 4
CIL_SOLVE_OK, CIL_SOLVE_NONFINITE, CIL_SOLVE_MAXSTEPS, CIL_SOLVE_FP32_FLOOR = 0, 1, 2, 3
CIL_POLISH_OFF, CIL_POLISH_FP64, CIL_POLISH_REFINE = 0, 1, 2
CIL_OPT_FORCE_EXACT_SUM = 1
CIL_OPT_QUAD_SHAPE = 2
CIL_OPT_BOOTSTRAP_GATHER = 3
CIL_OPT_GRAM_FLUSH = 4
CIL_OPT_GRAM_PIPELINE = 5
CIL_OPT_WAVE_PRIORITY = 6
CIL_OPT_POLISH_SEPARATE = 7
CIL_OPT_SYNC_SPIN_US = 8
CIL_OPT_STAT_DEVICE_RADII = 9
CIL_QUAD_SHAPES = 4


class CilError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_strerror(code), code, msg))
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("L", ctypes.c_double),
                ("nu", ctypes.c_double * 2), ("p", ctypes.c_double * 4)]


# numpy view of a Problem array (same field order, sizes and offsets)
_PROBLEM_DTYPE = np.dtype([("n", np.int32), ("reserved", np.int32), ("L", np.float64), ("nu", np.float64, 2),
                           ("p", np.float64, 4)])


def _state_sizes(problems, B: int) -> np.ndarray:
    """Elements of each solve's state, 2 n^2 (a view of the array, no loop over ctypes fields)."""
    if B == 0:
        return np.zeros(0, dtype=np.int64)
    n = np.frombuffer(problems, dtype=_PROBLEM_DTYPE, count=B)["n"].astype(np.int64)
    return 2 * n * n


class Stepping(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("max_steps", ctypes.c_int64), ("tol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("path", ctypes.c_int32), ("polish", ctypes.c_int32),
                ("fp32_floor_ulps", ctypes.c_int32)]


class SolveReport(ctypes.Structure):
    _fields_ = [("steps_taken", ctypes.c_int64), ("steps_fp64", ctypes.c_int64),
                ("final_resid", ctypes.c_double), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# numpy view of a SolveReport array (same field order, sizes and offsets)
_REPORT_DTYPE = np.dtype([("steps_taken", np.int64), ("steps_fp64", np.int64), ("final_resid", np.float64),
                          ("status", np.int32), ("reserved", np.int32)])


def _reports(reps, B: int):
    a = np.frombuffer(reps, dtype=_REPORT_DTYPE, count=B) if B else np.zeros(0, dtype=_REPORT_DTYPE)
    return dict(steps_taken=a["steps_taken"].copy(), steps_fp64=a["steps_fp64"].copy(),
                final_resid=a["final_resid"].copy(), status=a["status"].copy())


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcil.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcil.so is not built: run `python -m paper_2203_14742_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.cil_strerror.restype = ctypes.c_char_p
        L.cil_strerror.argtypes = [ctypes.c_int]
        L.cil_last_error.restype = ctypes.c_char_p
        L.cil_homogeneous_state.argtypes = [ctypes.c_int, vp, vp]
        L.cil_simulate_patterns.argtypes = [ctypes.c_int, ctypes.c_int, vp, i32, vp, vp, vp, vp, vp]
        L.cil_simulate_patterns_sbdf2.argtypes = [ctypes.c_int, ctypes.c_int, vp, i32, vp, vp, vp, vp, vp]
        L.cil_features.argtypes = [vp, i64, vp, i64, i64, ctypes.c_int, vp, i32, vp, vp, vp]
        L.cil_pair_bins.argtypes = [vp, i64, vp, i64, i64, ctypes.c_int, vp, i32, vp, vp, vp]
        L.cil_distance_range.argtypes = [vp, i64, vp, i64, i64, ctypes.c_int, i32, vp, vp, vp]
        L.cil_canonical_d2.argtypes = [vp, i64, vp, i64, i64, ctypes.c_int, vp, vp, i64, vp, vp]
        L.cil_radii.argtypes = [dbl, dbl, i32, i32, vp]
        L.cil_pair_bins_adaptive.argtypes = [vp, i64, vp, i64, i64, ctypes.c_int, i32, i32, i32, vp, vp, vp, vp, vp,
                                             vp]
        L.cil_approx_d2.argtypes = [vp, i64, vp, i64, i64, ctypes.c_int, vp, vp, vp]
        L.cil_approx_d2.restype = ctypes.c_int
        L.cil_last_distance_stats.argtypes = [vp, vp, vp]
        L.cil_bootstrap_features.argtypes = [vp, i64, i64, i32, vp, i32, vp, i32, i32, vp, vp, vp]
        L.cil_bootstrap_features_noalloc.argtypes = [vp, i64, i64, i32, vp, i32, vp, i32, i32, vp, vp, vp]
        L.cil_gaussian_loglik.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.cil_statistic_adaptive.argtypes = [vp, i64, vp, i64, i64, ctypes.c_int, i32, i32, vp, i32, vp, i32, i32,
                                             vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.cil_statistic_adaptive.restype = ctypes.c_int
        L.cil_set_option.argtypes = [i32, i64]
        L.cil_profile.argtypes = [i32]
        L.cil_profile_read.argtypes = [ctypes.c_char_p, vp, vp]
        L.cil_profile_names.argtypes = [vp, i64]
        L.cil_minmax_scale.argtypes = [vp, i64, i32, ctypes.c_int, vp, vp]
        L.cil_augment_patterns.argtypes = [vp, i64, i32, dbl, ctypes.c_int, vp, vp]
        L.cil_pair_maxabs.argtypes = [vp, i64, vp, i64, i64, ctypes.c_int, vp, i32, vp, vp]
        L.cil_combine_segments.argtypes = [vp, i64, i32, i32, vp, vp]
        L.cil_value_range.argtypes = [vp, i64, vp, vp, vp]
        L.cil_bin_values.argtypes = [vp, i64, vp, i32, vp, vp, vp]
        L.cil_sim_plan_create.argtypes = [ctypes.c_int, ctypes.c_int, vp, i32, vp, vp, vp, vp, vp]
        L.cil_sim_plan_tune.argtypes = [vp, i64, vp]
        L.cil_sim_plan_launch.argtypes = [vp, vp]
        L.cil_sim_plan_report.argtypes = [vp, vp, vp]
        L.cil_sim_plan_groups.argtypes = [vp]
        L.cil_sim_plan_group_info.argtypes = [vp, i32, vp, vp, vp, vp]
        L.cil_sim_plan_destroy.argtypes = [vp]
        for name in ("cil_homogeneous_state", "cil_simulate_patterns", "cil_features", "cil_pair_bins",
                     "cil_distance_range", "cil_canonical_d2", "cil_radii", "cil_last_distance_stats",
                     "cil_bootstrap_features", "cil_bootstrap_features_noalloc", "cil_gaussian_loglik", "cil_set_option", "cil_shutdown",
                     "cil_profile", "cil_profile_read", "cil_profile_names", "cil_sim_plan_create",
                     "cil_sim_plan_tune", "cil_sim_plan_launch", "cil_sim_plan_report", "cil_sim_plan_groups",
                     "cil_sim_plan_group_info", "cil_sim_plan_destroy", "cil_minmax_scale", "cil_augment_patterns",
                     "cil_pair_maxabs", "cil_combine_segments", "cil_value_range", "cil_bin_values"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().cil_strerror(code).decode()
    except Exception:
        return "error"


def _check(rc: int):
    if rc != CIL_OK:
        raise CilError(rc, lib().cil_last_error().decode())


def _stream(t=None):
    import torch
    dev = t.device if t is not None else torch.device("cuda", torch.cuda.current_device())
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _prec(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return CIL_FP64
    if t.dtype == torch.float32:
        return CIL_FP32
    raise TypeError("patterns must be float32 or float64, got %s" % t.dtype)


def _dev(t, what: str):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return ctypes.c_void_p(t.data_ptr())


def _arr(x, dtype):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


# ------------------------------------------------------------------ models

def cil_homogeneous_state(model: int, p: Sequence[float]):
    pp = np.zeros(4)
    pp[: len(p)] = p
    out = np.zeros(2)
    _check(lib().cil_homogeneous_state(model, pp.ctypes.data, out.ctypes.data))
    return float(out[0]), float(out[1])


def make_problems(n, L, nu, p, count: int | None = None):
    """Problem array; each argument a scalar/tuple for all solves or one row per solve."""
    n_arr = np.atleast_1d(np.asarray(n, dtype=np.int64))
    L_arr = np.atleast_1d(np.asarray(L, dtype=np.float64))
    nu_arr = np.atleast_2d(np.asarray(nu, dtype=np.float64))
    p_arr = np.atleast_2d(np.asarray(p, dtype=np.float64))
    B = count or max(n_arr.size, L_arr.size, nu_arr.shape[0], p_arr.shape[0])
    if nu_arr.shape[1] != 2:
        raise ValueError("nu needs two diffusion coefficients per solve")
    probs = (Problem * B)()
    if B == 0:
        return probs
    rows = np.arange(B)
    a = np.zeros(B, dtype=_PROBLEM_DTYPE)
    a["n"] = n_arr[rows % n_arr.size]
    a["L"] = L_arr[rows % L_arr.size]
    a["nu"] = nu_arr[rows % nu_arr.shape[0], :2]
    k = min(4, p_arr.shape[1])
    a["p"][:, :k] = p_arr[rows % p_arr.shape[0], :k]
    ctypes.memmove(probs, a.ctypes.data, a.nbytes)
    return probs


def cil_simulate_patterns(model: int, state, problems, dt: float, max_steps: int, tol: float = 0.0,
                          check_every: int = 1, path: int = CIL_PATH_AUTO, polish: int = 1,
                          fp32_floor_ulps: int = 0, offsets=None, raise_on_nonfinite: bool = True,
                          scheme: str = "euler"):
    """Run the solves in place on ``state`` (float32/float64 device tensor).
    scheme "euler": IMEX Euler (cil_simulate_patterns); "sbdf2": the
    second-order IMEX stepper (cil_simulate_patterns_sbdf2; with the AUTO
    path the fused line kernel k_fused_sbdf2 runs n = 32 in FP32 and FP64 and
    n = 64 in FP32, the plain back-end every other side; FP32 with polish=0
    only).
    Returns a dict of numpy arrays: steps_taken, steps_fp64, final_resid, status."""
    if scheme not in ("euler", "sbdf2"):
        raise ValueError("unknown scheme %r" % (scheme,))
    B = len(problems)
    st = Stepping(dt=dt, max_steps=int(max_steps), tol=tol, check_every=int(check_every), path=int(path),
                  polish=int(polish), fp32_floor_ulps=int(fp32_floor_ulps))
    reps = (SolveReport * max(B, 1))()
    offs = None
    sizes = _state_sizes(problems, B)
    if offsets is not None:
        offs = _arr(offsets, np.int64)
        need = int((offs + sizes).max()) if B else 0
    else:
        need = int(sizes.sum())
    if state.numel() < need:
        raise ValueError("state holds %d elements, the solves need %d" % (state.numel(), need))
    fn = lib().cil_simulate_patterns if scheme == "euler" else lib().cil_simulate_patterns_sbdf2
    rc = fn(model, _prec(state), ctypes.cast(problems, ctypes.c_void_p), B, _dev(state, "state"),
            None if offs is None else offs.ctypes.data, ctypes.byref(st), ctypes.cast(reps, ctypes.c_void_p),
            _stream(state))
    out = _reports(reps, B)
    if rc == CIL_ENONFINITE and not raise_on_nonfinite:
        return out
    _check(rc)
    return out


class SimPlan:
    """A batch of fused solves bound to ``state`` and to one HIP graph
    (``cil_sim_plan_*``).  ``launch()`` replays it on the current stream: every
    solve restarts at step 0 from what ``state`` holds.  The tensor must stay
    alive (and in place) while the plan lives."""

    def __init__(self, model: int, state, problems, dt: float, max_steps: int, tol: float = 0.0,
                 check_every: int = 1, path: int = CIL_PATH_AUTO, fp32_floor_ulps: int = 0, offsets=None):
        self.B = len(problems)
        self.state = state
        self._h = ctypes.c_void_p()
        stp = Stepping(dt=dt, max_steps=int(max_steps), tol=tol, check_every=int(check_every), path=int(path),
                       polish=0, fp32_floor_ulps=int(fp32_floor_ulps))
        sizes = _state_sizes(problems, self.B)
        offs = None
        if offsets is not None:
            offs = _arr(offsets, np.int64)
            need = int((offs + sizes).max()) if self.B else 0
        else:
            need = int(sizes.sum())
        if state.numel() < need:
            raise ValueError("state holds %d elements, the solves need %d" % (state.numel(), need))
        self._offs = offs
        _check(lib().cil_sim_plan_create(model, _prec(state), ctypes.cast(problems, ctypes.c_void_p), self.B,
                                         _dev(state, "state"), None if offs is None else offs.ctypes.data,
                                         ctypes.byref(stp), _stream(state), ctypes.byref(self._h)))

    def tune(self, steps: int = 100):
        """Autotune the code shape per grid side; returns group_info()."""
        _check(lib().cil_sim_plan_tune(self._h, int(steps), _stream(self.state)))
        return self.group_info()

    def group_info(self):
        out = []
        for g in range(_nonneg(lib().cil_sim_plan_groups(self._h))):
            n, c, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            ms = (ctypes.c_double * CIL_QUAD_SHAPES)()
            _check(lib().cil_sim_plan_group_info(self._h, g, ctypes.byref(n), ctypes.byref(c), ctypes.byref(s), ms))
            out.append(dict(n=n.value, count=c.value, shape=s.value, tuned_ms=list(ms)))
        return out

    def launch(self):
        _check(lib().cil_sim_plan_launch(self._h, _stream(self.state)))

    def report(self, raise_on_nonfinite: bool = True):
        reps = (SolveReport * self.B)()
        rc = lib().cil_sim_plan_report(self._h, ctypes.cast(reps, ctypes.c_void_p), _stream(self.state))
        out = _reports(reps, self.B)
        del out["steps_fp64"]
        if rc == CIL_ENONFINITE and not raise_on_nonfinite:
            return out
        _check(rc)
        return out

    def close(self):
        if self._h:
            _check(lib().cil_sim_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _nonneg(rc: int) -> int:
    if rc < 0:
        _check(rc)
    return rc


# ------------------------------------------------------- CIL statistic

def _sets(A, B):
    if A.dtype != B.dtype:
        raise TypeError("sets must share a dtype")
    A2 = A.reshape(A.shape[0], int(np.prod(A.shape[1:])))
    B2 = B.reshape(B.shape[0], int(np.prod(B.shape[1:])))
    if A2.shape[1] != B2.shape[1]:
        raise ValueError("sets must share the pattern dimension")
    return A2, B2


def cil_features(A, B, radii):
    """counts[m] = #{(i,j) : D(A_i,B_j) < R_m^2} and y = counts / (nA nB)."""
    A2, B2 = _sets(A, B)
    r = _arr(radii, np.float64)
    counts = np.zeros(r.size, dtype=np.int64)
    y = np.zeros(r.size)
    _check(lib().cil_features(_dev(A2, "A"), A2.shape[0], _dev(B2, "B"), B2.shape[0], A2.shape[1], _prec(A2),
                              r.ctypes.data, r.size, counts.ctypes.data, y.ctypes.data, _stream(A2)))
    return counts, y


def cil_pair_bins(A, B, radii, bins=None, want_counts: bool = True):
    import torch
    A2, B2 = _sets(A, B)
    r = _arr(radii, np.float64)
    if bins is None:
        bins = torch.empty((A2.shape[0], B2.shape[0]), dtype=torch.uint8, device=A2.device)
    counts = np.zeros(r.size, dtype=np.int64)
    _check(lib().cil_pair_bins(_dev(A2, "A"), A2.shape[0], _dev(B2, "B"), B2.shape[0], A2.shape[1], _prec(A2),
                               r.ctypes.data, r.size, _dev(bins, "bins"),
                               counts.ctypes.data if want_counts else None, _stream(A2)))
    return bins, counts


def cil_pair_bins_adaptive(A, B, M: int, law: int = 0, bins=None, want_bins: bool = True,
                           exclude_diagonal: bool = False):
    """Range, radii and bins from one fast pass.  Returns (d2min, d2max,
    radii host float64[M], bins uint8 [nA, nB] device tensor or None, counts int64[M])."""
    import torch
    A2, B2 = _sets(A, B)
    if want_bins and bins is None:
        bins = torch.empty((A2.shape[0], B2.shape[0]), dtype=torch.uint8, device=A2.device)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    radii = np.zeros(M, dtype=np.float64)
    counts = np.zeros(M, dtype=np.int64)
    _check(lib().cil_pair_bins_adaptive(_dev(A2, "A"), A2.shape[0], _dev(B2, "B"), B2.shape[0], A2.shape[1],
                                        _prec(A2), int(exclude_diagonal), M, law, ctypes.byref(lo), ctypes.byref(hi),
                                        radii.ctypes.data,
                                        _dev(bins, "bins") if want_bins else None, counts.ctypes.data, _stream(A2)))
    return lo.value, hi.value, radii, (bins if want_bins else None), counts


def cil_distance_range(A, B, exclude_diagonal: bool = False):
    A2, B2 = _sets(A, B)
    lo = ctypes.c_double()
    hi = ctypes.c_double()
    _check(lib().cil_distance_range(_dev(A2, "A"), A2.shape[0], _dev(B2, "B"), B2.shape[0], A2.shape[1],
                                    _prec(A2), int(bool(exclude_diagonal)), ctypes.byref(lo), ctypes.byref(hi),
                                    _stream(A2)))
    return lo.value, hi.value


def cil_canonical_d2(A, B, ia, jb):
    import torch
    A2, B2 = _sets(A, B)
    ia = ia.to(device=A2.device, dtype=torch.int64).contiguous()
    jb = jb.to(device=A2.device, dtype=torch.int64).contiguous()
    out = torch.empty(ia.numel(), dtype=torch.float64, device=A2.device)
    _check(lib().cil_canonical_d2(_dev(A2, "A"), A2.shape[0], _dev(B2, "B"), B2.shape[0], A2.shape[1], _prec(A2),
                                  _dev(ia, "ia"), _dev(jb, "jb"), ia.numel(), _dev(out, "d2"), _stream(A2)))
    return out


def cil_approx_d2(A, B):
    """(fast-pass squared distances, their error bounds) as [nA, nB] float64 device tensors."""
    import torch
    A2, B2 = _sets(A, B)
    d2 = torch.empty((A2.shape[0], B2.shape[0]), dtype=torch.float64, device=A2.device)
    eps = torch.empty_like(d2)
    _check(lib().cil_approx_d2(_dev(A2, "A"), A2.shape[0], _dev(B2, "B"), B2.shape[0], A2.shape[1], _prec(A2),
                               _dev(d2, "d2"), _dev(eps, "eps"), _stream(A2)))
    return d2, eps


def cil_radii(d2min: float, d2max: float, M: int, law: int = 0):
    out = np.zeros(M)
    _check(lib().cil_radii(float(d2min), float(d2max), int(M), int(law), out.ctypes.data))
    return out


def cil_last_distance_stats():
    v = np.zeros(3, dtype=np.int64)
    _check(lib().cil_last_distance_stats(v.ctypes.data, v[1:].ctypes.data, v[2:].ctypes.data))
    return dict(pairs=int(v[0]), rechecked=int(v[1]), exact_fallbacks=int(v[2]))


def cil_bootstrap_features(bins, idxA, idxB, M: int, want_counts: bool = True):
    """Returns (Ycount int64 [n_boot, M] or None, Y float64 [n_boot, M]) device tensors."""
    import torch
    nA, nB = bins.shape
    idxA = idxA.to(device=bins.device, dtype=torch.int32).contiguous()
    idxB = idxB.to(device=bins.device, dtype=torch.int32).contiguous()
    n_boot, kA = idxA.shape
    kB = idxB.shape[1]
    if idxB.shape[0] != n_boot:
        raise ValueError("index lists must have the same number of resamples")
    Y = torch.empty((n_boot, M), dtype=torch.float64, device=bins.device)
    Yc = torch.empty((n_boot, M), dtype=torch.int64, device=bins.device) if want_counts else None
    _check(lib().cil_bootstrap_features(_dev(bins, "bins"), nA, nB, M, _dev(idxA, "idxA"), kA, _dev(idxB, "idxB"),
                                        kB, n_boot, None if Yc is None else _dev(Yc, "Ycount"), _dev(Y, "Y"),
                                        _stream(bins)))
    return Yc, Y


def cil_gaussian_loglik(Y, y_obs):
    """Y [P, n_boot, M] (or [n_boot, M]) and y_obs [P, M] float64 device tensors."""
    import torch
    if Y.dim() == 2:
        Y = Y.unsqueeze(0)
        y_obs = y_obs.reshape(1, -1)
    Y = Y.contiguous()
    y_obs = y_obs.to(dtype=torch.float64).contiguous()
    P, n, M = Y.shape
    f = torch.empty(P, dtype=torch.float64, device=Y.device)
    ll = torch.empty(P, dtype=torch.float64, device=Y.device)
    me = torch.empty(P, dtype=torch.int32, device=Y.device)
    stt = torch.empty(P, dtype=torch.int32, device=Y.device)
    _check(lib().cil_gaussian_loglik(_dev(Y, "Y"), P, n, M, _dev(y_obs, "y_obs"), _dev(f, "f"), _dev(ll, "loglik"),
                                     _dev(me, "m_eff"), _dev(stt, "status"), _stream(Y)))
    return f, ll, me, stt


def cil_statistic_adaptive(A, B, M: int, idxA, idxB, law: int = 0, bins=None, Y=None, y_obs=None):
    """Alg. 2bst in one call: range, radii, bins and counts of the cross pairs,
    the bootstrap vectors Y, the observed vector y_obs = counts / (nA nB) and
    its Gaussian log-likelihood.  Returns (d2min, d2max, radii host float64[M],
    counts int64[M], bins, Y, y_obs, (f, loglik, m_eff, status)) with device
    tensors for bins [nA, nB] uint8, Y [n_boot, M], y_obs [M] and the
    likelihood outputs [1]."""
    import torch
    A2, B2 = _sets(A, B)
    nA, nB = A2.shape[0], B2.shape[0]
    dev = A2.device
    idxA = idxA.to(device=dev, dtype=torch.int32).contiguous()
    idxB = idxB.to(device=dev, dtype=torch.int32).contiguous()
    n_boot, kA = idxA.shape
    kB = idxB.shape[1]
    if idxB.shape[0] != n_boot:
        raise ValueError("index lists must have the same number of resamples")
    if bins is None:
        bins = torch.empty((nA, nB), dtype=torch.uint8, device=dev)
    if Y is None:
        Y = torch.empty((n_boot, M), dtype=torch.float64, device=dev)
    if y_obs is None:
        y_obs = torch.empty(M, dtype=torch.float64, device=dev)
    f = torch.empty(1, dtype=torch.float64, device=dev)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    me = torch.empty(1, dtype=torch.int32, device=dev)
    stt = torch.empty(1, dtype=torch.int32, device=dev)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    radii = np.zeros(M, dtype=np.float64)
    counts = np.zeros(M, dtype=np.int64)
    _check(lib().cil_statistic_adaptive(_dev(A2, "A"), nA, _dev(B2, "B"), nB, A2.shape[1], _prec(A2), M, law,
                                        _dev(idxA, "idxA"), kA, _dev(idxB, "idxB"), kB, n_boot, ctypes.byref(lo),
                                        ctypes.byref(hi), radii.ctypes.data, counts.ctypes.data, _dev(bins, "bins"),
                                        _dev(Y, "Y"), _dev(y_obs, "y_obs"), _dev(f, "f"), _dev(ll, "loglik"),
                                        _dev(me, "m_eff"), _dev(stt, "status"), _stream(A2)))
    return lo.value, hi.value, radii, counts, bins, Y, y_obs, (f, ll, me, stt)


# ------------------------------------------------ further features (Sec. 3.1)

def cil_minmax_scale(patterns, n: int, out=None):
    """Per pattern and species: (s - min) / (max - min) (FP64, rounded once)."""
    import torch
    if out is None:
        out = torch.empty_like(patterns)
    count = patterns.numel() // (2 * n * n)
    _check(lib().cil_minmax_scale(_dev(patterns, "patterns"), count, n, _prec(patterns), _dev(out, "out"),
                                  _stream(patterns)))
    return out


def augmented_dim(n: int) -> int:
    return 2 * n * n + 4 * n * (n - 1)


def cil_augment_patterns(patterns, n: int, L: float):
    """[s | D_x s | D_y s] per pattern (forward differences, h = L / (n - 1))."""
    import torch
    count = patterns.numel() // (2 * n * n)
    out = torch.empty((count, augmented_dim(n)), dtype=patterns.dtype, device=patterns.device)
    _check(lib().cil_augment_patterns(_dev(patterns, "patterns"), count, n, float(L), _prec(patterns),
                                      _dev(out, "out"), _stream(patterns)))
    return out


def cil_pair_maxabs(A, B, seg_end):
    """D[i, j, s] = max over segment s of |A_ik - B_jk| (FP64, exact max rounded once)."""
    import torch
    A2, B2 = _sets(A, B)
    se = _arr(seg_end, np.int64)
    D = torch.empty((A2.shape[0], B2.shape[0], se.size), dtype=torch.float64, device=A2.device)
    _check(lib().cil_pair_maxabs(_dev(A2, "A"), A2.shape[0], _dev(B2, "B"), B2.shape[0], A2.shape[1], _prec(A2),
                                 se.ctypes.data, se.size, _dev(D, "D"), _stream(A2)))
    return D


def cil_combine_segments(D, mode: int):
    """max (mode 0) or left-to-right sum (mode 1) over the last axis of D."""
    import torch
    nseg = D.shape[-1]
    out = torch.empty(D.shape[:-1], dtype=torch.float64, device=D.device)
    _check(lib().cil_combine_segments(_dev(D, "D"), out.numel(), nseg, int(mode), _dev(out, "out"), _stream(D)))
    return out


def cil_value_range(V):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().cil_value_range(_dev(V, "V"), V.numel(), ctypes.byref(lo), ctypes.byref(hi), _stream(V)))
    return lo.value, hi.value


def cil_bin_values(V, radii, want_bins: bool = True):
    """bins = #{m : V < R_m} (uint8, V's shape), counts[m] = #{bins >= m + 1}."""
    import torch
    r = _arr(radii, np.float64)
    bins = torch.empty(V.shape, dtype=torch.uint8, device=V.device) if want_bins else None
    counts = np.zeros(r.size, dtype=np.int64)
    _check(lib().cil_bin_values(_dev(V, "V"), V.numel(), r.ctypes.data, r.size,
                                None if bins is None else _dev(bins, "bins"), counts.ctypes.data, _stream(V)))
    return bins, counts


def cil_set_option(option: int, value: int):
    _check(lib().cil_set_option(int(option), int(value)))


def cil_profile(enable):
    """False/0: off; True/1: every hot kernel; 2: the fused stepper kernels only."""
    _check(lib().cil_profile(2 if enable == 2 else int(bool(enable))))


def cil_profile_read(name: str):
    """(number of timed launches, total milliseconds) for one kernel name."""
    c = ctypes.c_int64()
    t = ctypes.c_double()
    _check(lib().cil_profile_read(name.encode(), ctypes.byref(c), ctypes.byref(t)))
    return int(c.value), float(t.value)


def cil_profile_names():
    buf = ctypes.create_string_buffer(4096)
    _check(lib().cil_profile_names(ctypes.cast(buf, ctypes.c_void_p), 4096))
    s = buf.value.decode()
    return s.split(",") if s else []


def cil_shutdown():
    _check(lib().cil_shutdown())
