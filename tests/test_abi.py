"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/cil.h declares, and its host-only functions and argument
validation behave as documented."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2203_14742_amd as cil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cil.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cil_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 13
    L = cil.lib()
    for n in names:
        assert hasattr(L, n), n


def test_header_is_plain_c():
    hdr = os.path.join(ROOT, "include", "cil.h")
    import subprocess
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", hdr],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_strerror_and_codes():
    L = cil.lib()
    assert L.cil_strerror(0) == b"success"
    assert L.cil_strerror(-1) == b"invalid argument"
    assert L.cil_strerror(-5).startswith(b"covariance")


def test_homogeneous_state_matches_oracle(oracle_mod):
    o = oracle_mod
    for model, p in [(0, (1.0, 10.0, 1.0)), (1, (0.5, 1.0)), (2, (0.5, 1.0)), (3, (4.5, 6.96)), (3, (3.0, 9.0))]:
        assert cil.cil_homogeneous_state(model, p) == o.homogeneous_state(model, p)
    with pytest.raises(cil.CilError):
        cil.cil_homogeneous_state(3, (0.0, 1.0))


@pytest.mark.parametrize("law", ["power", "linear"])
def test_radii_bit_identical_to_oracle(oracle_mod, law):
    o = oracle_mod
    g = np.random.default_rng(0)
    for _ in range(50):
        lo = float(g.uniform(0.1, 100.0))
        hi = lo * float(g.uniform(1.01, 1e4))
        M = int(g.integers(1, 40))
        a = cil.cil_radii(lo, hi, M, 0 if law == "power" else 1)
        b = o.radii_ladder(lo, hi, M, law)
        assert np.array_equal(a, b)


def test_radii_rejects_degenerate_range():
    with pytest.raises(cil.CilError) as e:
        cil.cil_radii(4.0, 4.0, 5)
    assert e.value.code == cil.CIL_EINVAL
    with pytest.raises(cil.CilError):
        cil.cil_radii(0.0, 4.0, 5)


def _simulate_raw(probs, stepping, B=None, state=1, entry="cil_simulate_patterns"):
    L = cil.lib()
    B = len(probs) if B is None else B
    return getattr(L, entry)(0, 0, ctypes.cast(probs, ctypes.c_void_p), B,
                             ctypes.c_void_p(state), None, ctypes.byref(stepping), None, None)


def test_simulate_argument_validation_before_device():
    """Bad arguments are rejected with CIL_EINVAL before any device work."""
    good = cil.Stepping(dt=0.01, max_steps=10, tol=0.0, check_every=1, path=0, polish=1, fp32_floor_ulps=0)
    probs = cil.make_problems(1, 1.0, (0.1, 0.1), (1.0, 1.0, 1.0))      # n = 1 < 2
    assert _simulate_raw(probs, good) == cil.CIL_EINVAL
    assert b"n = 1" in cil.lib().cil_last_error()
    probs = cil.make_problems(8, 1.0, (0.1, 0.1), (1.0, 1.0, 1.0))
    for field, val in (("dt", 0.0), ("dt", -1.0), ("max_steps", -1), ("check_every", 0), ("path", 7), ("polish", 3),
                       ("polish", -1)):
        st = cil.Stepping(dt=0.01, max_steps=10, tol=0.0, check_every=1, path=0, polish=1, fp32_floor_ulps=0)
        setattr(st, field, val)
        assert _simulate_raw(probs, st) == cil.CIL_EINVAL, field
    assert _simulate_raw(probs, good, state=0) == cil.CIL_EINVAL                 # null state
    probs_badL = cil.make_problems(8, -1.0, (0.1, 0.1), (1.0, 1.0, 1.0))
    assert _simulate_raw(probs_badL, good) == cil.CIL_EINVAL
    assert _simulate_raw(probs, good, B=0) == cil.CIL_OK                          # empty batch


def test_second_order_entry_validates_like_the_euler_one():
    """The second-order entry point takes the same checks before any device
    work; the binding rejects an unknown scheme before calling the library."""
    good = cil.Stepping(dt=0.01, max_steps=10, tol=0.0, check_every=1, path=0, polish=0, fp32_floor_ulps=0)
    e = "cil_simulate_patterns_sbdf2"
    assert _simulate_raw(cil.make_problems(1, 1.0, (0.1, 0.1), (1.0, 1.0, 1.0)), good, entry=e) == cil.CIL_EINVAL
    probs = cil.make_problems(8, 1.0, (0.1, 0.1), (1.0, 1.0, 1.0))
    for field, val in (("dt", 0.0), ("max_steps", -1), ("check_every", 0), ("path", 7), ("polish", 3)):
        st = cil.Stepping(dt=0.01, max_steps=10, tol=0.0, check_every=1, path=0, polish=0, fp32_floor_ulps=0)
        setattr(st, field, val)
        assert _simulate_raw(probs, st, entry=e) == cil.CIL_EINVAL, field
    assert _simulate_raw(probs, good, state=0, entry=e) == cil.CIL_EINVAL
    assert _simulate_raw(probs, good, B=0, entry=e) == cil.CIL_OK
    with pytest.raises(ValueError):
        cil.cil_simulate_patterns(0, None, probs, 0.01, 10, scheme="rk4")


def test_statistic_argument_validation():
    L = cil.lib()
    r = np.array([3.0, 2.0, 2.0])            # not strictly decreasing
    c = np.zeros(3, dtype=np.int64)
    rc = L.cil_features(ctypes.c_void_p(1), 4, ctypes.c_void_p(1), 4, 8, 0, r.ctypes.data, 3, c.ctypes.data,
                        None, None)
    assert rc == cil.CIL_EINVAL
    r = np.array([3.0, -2.0])
    assert L.cil_pair_bins(ctypes.c_void_p(1), 4, ctypes.c_void_p(1), 4, 8, 0, r.ctypes.data, 2, None, None,
                           None) == cil.CIL_EINVAL
    r = np.linspace(300, 1, 256)             # M > 255
    assert L.cil_pair_bins(ctypes.c_void_p(1), 4, ctypes.c_void_p(1), 4, 8, 0, r.ctypes.data, 256, None, None,
                           None) == cil.CIL_EINVAL
    lo, hi = ctypes.c_double(), ctypes.c_double()
    assert L.cil_distance_range(ctypes.c_void_p(1), 3, ctypes.c_void_p(1), 4, 8, 0, 1, ctypes.byref(lo),
                                ctypes.byref(hi), None) == cil.CIL_EINVAL       # diagonal needs nA == nB
    assert L.cil_gaussian_loglik(None, 1, 1, 4, None, None, None, None, None, None) == cil.CIL_EINVAL
    assert L.cil_gaussian_loglik(None, 1, 10, 65, None, None, None, None, None, None) == cil.CIL_EINVAL
    assert L.cil_bootstrap_features(None, 4, 4, 0, None, 1, None, 1, 1, None, None, None) == cil.CIL_EINVAL
    assert L.cil_set_option(99, 0) == cil.CIL_EINVAL
    for bad in (-1, 10000001):
        assert L.cil_set_option(cil.CIL_OPT_SYNC_SPIN_US, bad) == cil.CIL_EINVAL
    for good in (0, 200000):
        assert L.cil_set_option(cil.CIL_OPT_SYNC_SPIN_US, good) == cil.CIL_OK
    for bad in (-1, 3):
        assert L.cil_set_option(cil.CIL_OPT_STAT_DEVICE_RADII, bad) == cil.CIL_EINVAL
    for good in (0, 2, 1):
        assert L.cil_set_option(cil.CIL_OPT_STAT_DEVICE_RADII, good) == cil.CIL_OK
    # the one-call statistic checks its sizes before touching the device
    assert L.cil_statistic_adaptive(None, 0, None, 4, 8, cil.CIL_FP32, 3, 0, None, 1, None, 1, 2, None, None, None,
                                    None, None, None, None, None, None, None, None, None) == cil.CIL_EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(cil, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(cil, "_lib", None)
    with pytest.raises(ImportError):
        cil.lib()
