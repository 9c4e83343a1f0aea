"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, a textbook/library routine, an exact rational computation, an invariant
or a brute-force count.  No GPU.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import cil_synth as cs

FHN_P = (1.0, 10.0, 1.0)          # (mu, eps, alpha), Table exp1
FHN_NU = (0.05, 0.00028)
GM_P = (0.5, 1.0)                  # (mu_v, mu_w), Table exp1
GM_NU = (0.00025, 0.01)
BZ_P = (4.5, 6.96)                 # (A, B), Table exp1
BZ_NU = (0.0016, 0.0132)
GMS_P = (0.5, 1.0)                 # (a, b) of the source form
GMS_NU = (1.0, 100.0)


def lam_1d(n, L, k):
    h = L / (n - 1)
    return (4.0 / h ** 2) * math.sin(math.pi * k / (2 * n)) ** 2


# --------------------------------------------------------------------------
# Models and steady states (Sec. 4.1)

def test_steady_states_closed_form(oracle_mod):
    o = oracle_mod
    assert o.homogeneous_state(o.FHN, FHN_P) == (0.0, 0.0)
    assert o.homogeneous_state(o.GM, GM_P) == (2.0, 4.0)          # (mu_w/mu_v, mu_w/mu_v^2)
    v0, w0 = o.homogeneous_state(o.BRUSSELATOR, BZ_P)
    assert v0 == 4.5 and abs(w0 - 6.96 / 4.5) < 1e-15            # (A, B/A)
    assert o.homogeneous_state(o.GM_SOURCE, GMS_P) == (1.5, 2.25)


@pytest.mark.parametrize("model,p", [(0, FHN_P), (1, GM_P), (2, GMS_P), (3, BZ_P)])
def test_kinetics_vanish_at_steady_state(oracle_mod, model, p):
    o = oracle_mod
    v0, w0 = o.homogeneous_state(model, p)
    f, g = o.kinetics(model, p, v0, w0)
    assert abs(f) < 1e-14 and abs(g) < 1e-14


def test_kinetics_values(oracle_mod):
    """Spot values of the reaction terms written out from Sec. 4.1."""
    o = oracle_mod
    assert o.kinetics(o.FHN, (2.0, 3.0, 0.5), 0.4, -0.7) == pytest.approx(
        (3.0 * (-0.7 - 0.5 * 0.4), -0.4 + 2.0 * -0.7 + 0.343), rel=1e-15)
    assert o.kinetics(o.GM, (0.5, 1.0), 1.2, 0.8) == pytest.approx(
        (-0.6 + 1.44 / 0.8, -0.8 + 1.44), rel=1e-15)
    assert o.kinetics(o.BRUSSELATOR, (4.5, 6.96), 1.1, 2.0) == pytest.approx(
        (4.5 - 7.96 * 1.1 + 1.21 * 2.0, 6.96 * 1.1 - 1.21 * 2.0), rel=1e-15)


@pytest.mark.parametrize("model,p,nu", [(0, FHN_P, FHN_NU), (1, GM_P, GM_NU), (2, GMS_P, GMS_NU)])
def test_P1_homogeneous_state_stays_fixed(oracle_mod, model, p, nu):
    o = oracle_mod
    n = 12
    v0, w0 = o.homogeneous_state(model, p)
    st = np.empty((1, 2, n, n))
    st[0, 0] = v0
    st[0, 1] = w0
    out, steps, res, status = o.imex_run(model, p, nu, n, 1.0, 0.05, 40, state=st)
    assert status[0] == 0 and steps[0] == 40
    assert np.abs(out[0, 0] - v0).max() <= 2e-13 * max(1.0, abs(v0))     # rounding drift only
    assert np.abs(out[0, 1] - w0).max() <= 2e-13 * max(1.0, abs(w0))
    assert res[0] <= 1e-12


# --------------------------------------------------------------------------
# Operator and implicit solve (App. B.1.1)

@pytest.mark.parametrize("n", [5, 8, 13])
def test_banded_cholesky_matches_dense_solve(oracle_mod, n):
    """The banded Cholesky solve agrees with a dense LAPACK solve of the
    stencil matrix assembled here from the ghost-copy rule."""
    o = oracle_mod
    L, dt, nu = 1.0, 0.02, 0.3
    h = L / (n - 1)
    N = n * n
    A = np.eye(N)
    c = dt * nu / h ** 2
    for i in range(n):
        for j in range(n):
            p = i * n + j
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:     # a ghost neighbour copies p itself
                    A[p, p] += c
                    A[p, ii * n + jj] -= c
    b = np.random.default_rng(n).standard_normal((n, n))
    x = o.implicit_diffusion(n, L, dt, nu, b)
    xr = np.linalg.solve(A, b.reshape(-1)).reshape(n, n)
    assert np.abs(x - xr).max() < 1e-13


@pytest.mark.parametrize("n", [7, 16, 33])
def test_cosine_modes_diagonalise_the_solve(oracle_mod, n):
    o = oracle_mod
    b = np.random.default_rng(7 + n).standard_normal((n, n))
    x1 = o.implicit_diffusion(n, 2.0, 0.1, 0.02, b)
    x2 = o.dct_modes_diffusion(n, 2.0, 0.1, 0.02, b)
    assert np.abs(x1 - x2).max() < 1e-13


@pytest.mark.parametrize("n,k,l", [(16, 0, 3), (16, 5, 5), (32, 3, 8), (20, 19, 1)])
def test_P2_cosine_eigenmode_decay(oracle_mod, n, k, l):
    """Without kinetics a cosine mode decays by exactly (1 + dt nu Lambda_kl)^-s
    per species, Lambda_kl = (4/h^2)(sin^2(pi k/2n) + sin^2(pi l/2n))."""
    o = oracle_mod
    L, dt, steps = 1.0, 0.01, 25
    nu = (0.05, 0.002)
    mode = cs.cosine_mode(n, k, l)
    st = np.stack([mode, -2.0 * mode])[None]
    out, _, _, _ = o.imex_run(o.HEAT, (0.0,), nu, n, L, dt, steps, state=st)
    Lam = lam_1d(n, L, k) + lam_1d(n, L, l)
    for s, sign in ((0, 1.0), (1, -2.0)):
        amp = (1.0 + dt * nu[s] * Lam) ** (-steps)
        assert np.abs(out[0, s] - sign * amp * mode).max() < 1e-13 * max(1, abs(sign))


def test_mol_rhs_of_cosine_mode(oracle_mod):
    """Direct stencil: Lap_h of a cosine mode is -Lambda_kl times the mode."""
    o = oracle_mod
    n, L, k, l = 24, 3.0, 4, 9
    mode = cs.cosine_mode(n, k, l)
    st = np.stack([mode, mode])
    rhs = o.mol_rhs(o.HEAT, (0.0,), (1.0, 0.5), n, L, st)
    Lam = lam_1d(n, L, k) + lam_1d(n, L, l)
    assert np.abs(rhs[0] + Lam * mode).max() < 1e-10 * Lam
    assert np.abs(rhs[1] + 0.5 * Lam * mode).max() < 1e-10 * Lam


def _jacobian(model, p, v, w):
    """Jacobian of the kinetics at (v, w), derived by hand from Sec. 4.1."""
    if model == 0:
        mu, eps, alpha = p
        return np.array([[-eps * alpha, eps], [-1.0, mu - 3 * w * w]])
    if model == 1:
        mv, mw = p
        return np.array([[-mv + 2 * v / w, -v * v / (w * w)], [2 * v, -mw]])
    if model == 2:
        a, b = p
        return np.array([[-b + 2 * v / w, -v * v / (w * w)], [2 * v, -1.0]])
    if model == 3:
        A, B = p
        return np.array([[-(B + 1) + 2 * v * w, v * v], [B - 2 * v * w, -v * v]])
    raise ValueError


@pytest.mark.parametrize("model,p,nu,n,kl,L,dt,eps", [(0, FHN_P, FHN_NU, 32, (3, 8), 1.0, 0.01, 1e-6),
                                                      (1, GM_P, GM_NU, 32, (2, 7), 1.0, 0.01, 1e-6),
                                                      (2, GMS_P, GMS_NU, 64, (6, 11), 120.0, 0.2, 1e-7),
                                                      (2, GMS_P, GMS_NU, 32, (3, 5), 60.0, 0.2, 1e-7),
                                                      (3, BZ_P, BZ_NU, 32, (3, 10), 1.0, 0.01, 1e-6)])
def test_P3_linear_single_mode_growth(oracle_mod, model, p, nu, n, kl, L, dt, eps):
    """A small perturbation along one cosine mode and one eigenvector of the
    per-step amplification matrix G = (I + dt Lambda diag nu)^-1 (I + dt J)
    grows by exactly that eigenvalue per step (to first order).  The
    Gierer-Meinhardt source form runs on the stationarity workload's domain
    (L = 120, dt = 0.2) and on a half-size one; it grows faster per step, so it
    starts from a smaller perturbation eps."""
    o = oracle_mod
    steps = 60
    v0, w0 = o.homogeneous_state(model, p)
    J = _jacobian(model, p, v0, w0)
    Lam = lam_1d(n, L, kl[0]) + lam_1d(n, L, kl[1])
    G = np.linalg.solve(np.eye(2) + dt * Lam * np.diag(nu), np.eye(2) + dt * J)
    ev, V = np.linalg.eig(G)
    assert np.all(np.abs(ev.imag) == 0)
    i = int(np.argmax(ev.real))
    rho, e = ev[i].real, V[:, i].real
    assert rho > 1.0                               # the mode is Turing-unstable
    # every Jacobian entry moves the predicted growth well past the bar, so a
    # wrong partial derivative of the kinetics cannot pass
    for (r, c) in ((0, 0), (0, 1), (1, 0), (1, 1)):
        Jw = J.copy()
        Jw[r, c] *= 1.1
        Gw = np.linalg.solve(np.eye(2) + dt * Lam * np.diag(nu), np.eye(2) + dt * Jw)
        rw = np.abs(np.linalg.eigvals(Gw)).max()
        assert abs((rw / rho) ** steps - 1.0) > 1e-3
    # eps: small enough that the quadratic terms stay below the bar after
    # `steps` steps of growth, large enough that rounding of the base state
    # stays below it too
    mode = cs.cosine_mode(n, *kl)
    st = np.stack([v0 + eps * e[0] * mode, w0 + eps * e[1] * mode])[None]
    out, _, _, _ = o.imex_run(model, p, nu, n, L, dt, steps, state=st)
    dv = (out[0, 0] - v0) / (eps * e[0] * rho ** steps)
    dw = (out[0, 1] - w0) / (eps * e[1] * rho ** steps)
    big = np.abs(mode) > 0.3
    assert np.abs(dv[big] / mode[big] - 1).max() < 1e-5
    assert np.abs(dw[big] / mode[big] - 1).max() < 1e-5


def _ring_index(n):
    k = np.arange(n)
    return np.rint(np.hypot(k[:, None], k[None, :])).astype(int)


@pytest.mark.parametrize("model,p,nu,n,L,dt", [(0, FHN_P, FHN_NU, 32, 1.0, 0.01),
                                               (1, GM_P, GM_NU, 32, 1.0, 0.01),
                                               (2, GMS_P, GMS_NU, 64, 120.0, 0.2),
                                               (3, BZ_P, BZ_NU, 32, 1.0, 0.01)])
def test_P4_dominant_wavenumber_of_the_dispersion_relation(oracle_mod, model, p, nu, n, L, dt):
    """From small noise about the homogeneous state, the linear phase selects
    the wavenumber at which the dispersion relation of eq. (rdgen) linearised
    about that state peaks (Sec. 4.1, operator of App. B.1.1).

    Prediction, written in the test: per cosine mode (k, l) the growth per
    step is the spectral radius of G_kl = (I + dt Lambda_kl diag nu)^-1 (I + dt J);
    the radially averaged expected power after S steps is the ring mean of
    G's radius^(2S) (rings of integer |(k, l)|).  The continuous-time
    relation sigma(q) = max Re eig(J - q^2 diag nu) gives k* in length units,
    q* n h / pi in mode units.  The oracle's radially averaged DCT-II power of
    the deviation after S steps (8 seeds) must peak within one ring of both.
    S keeps the growth below 1e3 (amplitude 1e-3: still linear)."""
    o = oracle_mod
    import scipy.fft as sf
    v0, w0 = o.homogeneous_state(model, p)
    J = _jacobian(model, p, v0, w0)
    h = L / (n - 1)
    lam = np.array([lam_1d(n, L, k) for k in range(n)])
    rho = np.empty((n, n))
    for k in range(n):
        for l in range(n):
            G = np.linalg.solve(np.eye(2) + dt * (lam[k] + lam[l]) * np.diag(nu), np.eye(2) + dt * J)
            rho[k, l] = np.abs(np.linalg.eigvals(G)).max()
    assert rho[0, 0] <= 1.0 < rho.max()            # Turing: not unstable without diffusion (FHN: neutral)
    S = int(math.log(1e3) / math.log(rho.max()))
    ring = _ring_index(n)
    cnt = np.bincount(ring.ravel())
    pred = np.bincount(ring.ravel(), (rho ** (2 * S)).ravel()) / cnt
    ring_pred = int(np.argmax(pred))
    q = np.linspace(1e-4, math.pi / h, 40001)
    sig = np.array([np.linalg.eigvals(J - qq * qq * np.diag(nu)).real.max() for qq in q])
    ring_cont = int(round(q[int(np.argmax(sig))] * n * h / math.pi))
    st = cs.initial_conditions((v0, w0), n, 8, seed=5, law="additive_sym", delta=1e-6)
    out, _, _, _ = o.imex_run(model, p, nu, n, L, dt, S, state=st, nthreads=4)
    dev = out - np.array([v0, w0])[None, :, None, None]
    assert np.abs(dev).max() < 1e-2
    power = (sf.dctn(dev, type=2, norm="ortho", axes=(2, 3)) ** 2).sum(axis=(0, 1))
    avg = np.bincount(ring.ravel(), power.ravel()) / cnt
    avg[0] = 0.0
    ring_meas = int(np.argmax(avg))
    assert abs(ring_meas - ring_pred) <= 1, (ring_meas, ring_pred)
    assert abs(ring_meas - ring_cont) <= 1, (ring_meas, ring_cont)
    assert abs(ring_pred - ring_cont) <= 1, (ring_pred, ring_cont)


def test_two_oracle_solvers_part_under_pattern_selection(oracle_mod):
    """The fixed-step FitzHugh-Nagumo workload (32^2, dt = 0.01, 128 solves)
    run by the oracle's banded Cholesky solve and, in this test, by the dense
    cosine-mode solve of App. B.1.1's operator (the same IMEX-Euler step):
    both are FP64 and correct, yet while patterns select (Sec. 1) their
    last-bit differences grow by orders of magnitude.  They agree within
    1e-10 (relative to max|u|) at 1000 steps and part beyond it by 5000, so a
    1e-10 bar at 5000 steps measures the problem's conditioning, not a
    solver."""
    o = oracle_mod
    w = cs.WORKLOADS["fhn32_fixed5000"]
    n, L, dt, nu = w["n"], w["L"], w["dt"], w["nu"]
    mu, eps, alpha = w["params"]
    base = o.homogeneous_state(w["model"], w["params"])
    ics = np.concatenate([cs.initial_conditions(base, n, w["count"], seed=s, law=w["ic_law"]) for s in w["seeds"]])
    h = L / (n - 1)
    i = np.arange(n)
    V = np.cos(np.pi * np.arange(n)[:, None] * (i + 0.5) / n)
    V /= np.sqrt((V * V).sum(1, keepdims=True))
    lam = (4.0 / h ** 2) * np.sin(np.pi * i / (2 * n)) ** 2
    div = np.stack([1.0 / (1.0 + dt * nu[s] * (lam[:, None] + lam[None, :])) for s in range(2)])
    cos_st, ref, done, errs = ics.copy(), ics.copy(), 0, {}
    for upto in (1000, 5000):
        for _ in range(upto - done):
            v, u = cos_st[:, 0], cos_st[:, 1]
            r = np.stack([v + dt * (eps * (u - alpha * v)), u + dt * (-v + mu * u - u * u * u)], 1)
            cos_st = V.T @ ((V @ r @ V.T) * div) @ V
        ref, _, _, _ = o.imex_run(w["model"], w["params"], nu, n, L, dt, upto - done, 0.0, upto - done,
                                  state=ref, nthreads=8)
        done = upto
        errs[upto] = np.abs(cos_st - ref).max() / np.abs(ref).max()
    assert errs[1000] < 1e-10, errs
    assert errs[5000] > 1e-10, errs


def test_P8_converged_pattern_solves_the_stencil_system(oracle_mod):
    """At an IMEX-Euler fixed point the method-of-lines right-hand side
    (App. B.1.1, eq. MOLSystem) vanishes; at residual r it is O(r)."""
    o = oracle_mod
    n, L, dt = 32, 60.0, 0.2
    base = o.homogeneous_state(o.GM_SOURCE, GMS_P)
    st = cs.initial_conditions(base, n, 1, 11, law="multiplicative")
    out, steps, res, status = o.imex_run(o.GM_SOURCE, GMS_P, GMS_NU, n, L, dt, 20000, 1e-9, 5,
                                         state=st)
    assert status[0] == 0 and res[0] < 1e-9
    assert np.ptp(out[0, 0]) > 0.5                 # a non-trivial pattern formed
    rhs = o.mol_rhs(o.GM_SOURCE, GMS_P, GMS_NU, n, L, out[0])
    assert np.abs(rhs).max() < 2e-8


def test_P9_resume_is_bitwise(oracle_mod):
    o = oracle_mod
    n = 16
    st = cs.initial_conditions((0.0, 0.0), n, 2, 5, law="additive_sym")
    a, _, _, _ = o.imex_run(o.FHN, FHN_P, FHN_NU, n, 1.0, 0.01, 70, state=st.copy())
    b1, _, _, _ = o.imex_run(o.FHN, FHN_P, FHN_NU, n, 1.0, 0.01, 30, state=st.copy())
    b2, _, _, _ = o.imex_run(o.FHN, FHN_P, FHN_NU, n, 1.0, 0.01, 40, state=b1)
    assert np.array_equal(a, b2)


def test_stop_rule_and_status(oracle_mod):
    o = oracle_mod
    n = 16
    base = o.homogeneous_state(o.GM_SOURCE, GMS_P)
    st = cs.initial_conditions(base, n, 1, 2, law="multiplicative")
    _, steps, res, status = o.imex_run(o.GM_SOURCE, GMS_P, GMS_NU, n, 30.0, 0.2, 5000, 1e-6, 7,
                                       state=st.copy())
    assert status[0] == 0 and steps[0] % 7 == 0 and res[0] < 1e-6
    _, steps2, res2, status2 = o.imex_run(o.GM_SOURCE, GMS_P, GMS_NU, n, 30.0, 0.2, 10, 1e-12, 3,
                                          state=st.copy())
    assert status2[0] == o.SOLVE_MAXSTEPS and steps2[0] == 10
    bad = st.copy()
    bad[0, 1, 3, 3] = np.nan
    _, steps3, res3, status3 = o.imex_run(o.GM_SOURCE, GMS_P, GMS_NU, n, 30.0, 0.2, 10, 0.0, 4,
                                          state=bad)
    assert status3[0] == o.SOLVE_NONFINITE and steps3[0] == 4


# --------------------------------------------------------------------------
# Canonical distance and counts (Sec. 2.1, eq. eCDF)

def _exact_d2(a, b):
    """Exact rational sum of fl64(a_k - b_k)^2, rounded once (half-even)."""
    s = Fraction(0)
    for x, y in zip(np.asarray(a, np.float64), np.asarray(b, np.float64)):
        d = Fraction(float(x - y))
        s += d * d
    return float(s)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_canonical_distance_is_exactly_rounded(oracle_mod, dtype):
    o = oracle_mod
    g = np.random.default_rng(3)
    for trial in range(40):
        d = int(g.integers(1, 300))
        scale = 10.0 ** g.integers(-6, 7)
        a = (g.standard_normal(d) * scale).astype(dtype)
        b = (a + g.standard_normal(d) * scale * 10.0 ** g.integers(-7, 1)).astype(dtype)
        assert o.canonical_d2(a, b) == _exact_d2(a, b)


def test_canonical_distance_order_independent(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(4)
    a = g.standard_normal(5000)
    b = g.standard_normal(5000)
    perm = g.permutation(5000)
    assert o.canonical_d2(a, b) == o.canonical_d2(a[perm], b[perm])


def test_exact_sum_against_fsum(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(5)
    for _ in range(20):
        x = g.standard_normal(1000) * 10.0 ** g.integers(-20, 20, size=1000)
        assert o.exact_sum(x) == math.fsum(x)
    assert o.exact_sum(np.array([1.0, 1e100, 1.0, -1e100])) == 2.0
    assert o.exact_sum(np.array([1.0, 2.0 ** -53, 2.0 ** -105])) == 1.0 + 2.0 ** -52


def test_P5_brute_force_counts_with_ties(oracle_mod):
    """Integer patterns make every distance exact; integer radii (exact
    squares) placed exactly on distances check the strict '<' of eq. (eCDF)."""
    o = oracle_mod
    g = np.random.default_rng(6)
    A = g.integers(-3, 4, size=(9, 7)).astype(np.float64)
    B = g.integers(-3, 4, size=(11, 7)).astype(np.float64)
    B[0] = A[0] + np.array([3, 4, 0, 0, 0, 0, 0])          # D = 25
    B[1] = A[2] + np.array([0, 0, 4, 0, 0, 0, 0])          # D = 16
    B[2] = A[5] + np.array([2, 0, 0, 1, 0, 2, 0])          # D = 9
    D = o.pair_d2(A, B)
    brute = np.array([[int(((A[i] - B[j]) ** 2).sum()) for j in range(11)] for i in range(9)])
    assert np.array_equal(D, brute.astype(np.float64))
    radii = np.arange(12, 0, -1).astype(np.float64)         # 12, 11, ..., 1
    c = o.counts_from_d2(D, radii)
    for m, R in enumerate(radii):
        assert c[m] == sum(1 for i in range(9) for j in range(11) if brute[i, j] < int(R) ** 2)
    for R in (5, 4, 3):                                     # ties present and not counted
        assert (brute == R * R).any()
        assert o.counts_from_d2(D, [float(R)])[0] == int((brute < R * R).sum())


def test_P6_count_invariants(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(8)
    A = g.standard_normal((12, 30))
    B = g.standard_normal((10, 30))
    lo, hi = o.distance_range(A, B)
    radii = o.radii_ladder(lo, hi, 9)
    cAB, yAB = o.cil_vector(A, B, radii)
    cBA, yBA = o.cil_vector(B, A, radii)
    assert np.array_equal(cAB, cBA)                           # symmetric in the sets
    assert np.all(np.diff(cAB) <= 0)                          # non-increasing in m
    assert np.all((yAB >= 0) & (yAB <= 1))
    D = o.pair_d2(A, B)                                       # R_M sits on the smallest distance:
    assert cAB[-1] <= int((D <= lo * (1 + 2.0 ** -50)).sum())  # only pairs within rounding of it
    cbig, _ = o.cil_vector(A, B, [2 * math.sqrt(hi)])
    assert cbig[0] == 12 * 10                                 # radius above every distance
    cAA, _ = o.cil_vector(A, A, [1e-3])
    assert cAA[0] == 12                                       # only the zero self-distances


def test_bins_consistent_with_counts(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(9)
    A = g.standard_normal((15, 20))
    B = g.standard_normal((13, 20))
    D = o.pair_d2(A, B)
    radii = o.radii_ladder(D.min(), D.max(), 11)
    bins = o.bins_from_d2(D, radii)
    c = o.counts_from_d2(D, radii)
    for m in range(11):
        assert c[m] == int((bins >= m + 1).sum())


def test_radii_ladder(oracle_mod):
    o = oracle_mod
    r = o.radii_ladder(4.0, 400.0, 13)
    assert np.all(np.diff(r) < 0)
    b = (20.0 / 2.0) ** (1 / 13)
    assert r[0] == pytest.approx(20.0 / b, rel=1e-15)
    assert r[-1] == pytest.approx(2.0, rel=1e-14)
    lin = o.radii_ladder(4.0, 400.0, 9, law="linear")
    assert np.allclose(np.diff(lin), -(20.0 - 2.0) / 9, rtol=1e-13)
    with pytest.raises(ValueError):
        o.radii_ladder(5.0, 5.0, 4)


# --------------------------------------------------------------------------
# Bootstrap (Alg. 2bst / 3bst step 2)

def test_bootstrap_identity_resample_equals_full_vector(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(10)
    A = g.standard_normal((14, 25))
    B = g.standard_normal((9, 25))
    D = o.pair_d2(A, B)
    radii = o.radii_ladder(D.min(), D.max(), 7)
    c, y = o.cil_vector(A, B, radii)
    ia = np.stack([np.arange(14), g.permutation(14)]).astype(np.int32)
    ib = np.stack([np.arange(9), g.permutation(9)]).astype(np.int32)
    Yc, Y = o.bootstrap_vectors(D, ia, ib, radii)
    assert np.array_equal(Yc[0], c) and np.array_equal(Yc[1], c)
    assert np.array_equal(Y[0], y)
    # doubling every index leaves the vector unchanged and quadruples the counts
    Yc2, Y2 = o.bootstrap_vectors(D, np.concatenate([ia, ia], 1), np.concatenate([ib, ib], 1), radii)
    assert np.array_equal(Yc2, 4 * Yc) and np.array_equal(Y2, Y)
    # a resample made of one row of A sees only that row's distances
    one = np.full((1, 5), 3, dtype=np.int32)
    Yc3, _ = o.bootstrap_vectors(D, one, ib[:1], radii)
    assert np.array_equal(Yc3[0], 5 * o.counts_from_d2(D[3], radii))


def test_resample_synthetic_respects_alg3bst(oracle_mod):
    i1, i2, sub = cs.resample_synthetic(20, 4, 50, seed=1)
    for r in range(50):
        assert not set(i2[r]).intersection(set(i1[r]))      # s2 from the remaining patterns
    assert len(set(sub)) == sub.size == 16


# --------------------------------------------------------------------------
# Statistics and cost (eqs. cil:CF, cil:CF_synth)

def test_P7_mean_cov_cholesky_against_library(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(11)
    Y = g.standard_normal((300, 6)) @ g.standard_normal((6, 6))
    mu, S = o.mean_cov(Y)
    assert np.allclose(mu, Y.mean(0), rtol=0, atol=1e-14)
    assert np.allclose(S, np.cov(Y.T), rtol=1e-13, atol=1e-14)
    Lc = o.cholesky(S)
    assert np.allclose(Lc @ Lc.T, S, rtol=0, atol=1e-13)
    assert np.allclose(Lc, np.linalg.cholesky(S), rtol=1e-12, atol=1e-14)


def test_P7_cost_and_loglik(oracle_mod):
    from scipy.stats import multivariate_normal
    o = oracle_mod
    g = np.random.default_rng(12)
    Y = g.standard_normal((500, 5)) @ g.standard_normal((5, 5)) + 3.0
    y = Y.mean(0) + g.standard_normal(5) * 0.3
    r = o.gaussian_cost(Y, y)
    mu, S = np.mean(Y, 0), np.cov(Y.T)
    assert r["ok"] and r["m_eff"] == 5
    assert r["f"] == pytest.approx(float((y - mu) @ np.linalg.solve(S, y - mu)), rel=1e-11)
    assert r["loglik"] == pytest.approx(multivariate_normal(mu, S).logpdf(y), rel=1e-11)
    assert o.gaussian_cost(Y, mu)["f"] == pytest.approx(0.0, abs=1e-20)


def test_P7_diagonal_and_dropped_bins(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(13)
    Y = np.zeros((400, 4))
    Y[:, 0] = g.standard_normal(400) * 2.0
    Y[:, 2] = g.standard_normal(400) * 0.5 + 1.0
    Y[:, 1] = 1.0                    # constant bin (radius above every distance)
    Y[:, 3] = 0.0                    # empty bin (radius at the smallest distance)
    y = np.array([0.3, 1.0, 0.2, 0.0])
    r = o.gaussian_cost(Y, y)
    assert r["m_eff"] == 2 and list(r["keep"]) == [True, False, True, False]
    mu, S = o.mean_cov(Y)
    a, b, d = S[0, 0], S[0, 2], S[2, 2]
    x0, x1 = 0.3 - mu[0], 0.2 - mu[2]
    f2 = (d * x0 * x0 - 2 * b * x0 * x1 + a * x1 * x1) / (a * d - b * b)   # 2x2 inverse
    assert r["f"] == pytest.approx(f2, rel=1e-12)


def test_nonspd_covariance_reports_failure(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(14)
    z = g.standard_normal(100)
    for Y in (np.stack([z, 2 * z, g.standard_normal(100)], 1),      # rank-deficient
              np.stack([z, z, g.standard_normal(100)], 1),
              np.stack([z, g.standard_normal(100), z - 0.5], 1)):
        r = o.gaussian_cost(Y, np.zeros(3))
        assert not r["ok"] and math.isnan(r["f"])
    with pytest.raises(np.linalg.LinAlgError):
        o.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))          # indefinite


# ------------------------------------------------ further features (Sec. 3.1, Sec. 5)

def test_minmax_scale_pins(oracle_mod):
    """Sec. 5 normalisation: a hand example, invariance under a positive affine
    map of the data, the constant-species reading, range [0, 1] attained."""
    o = oracle_mod
    x = np.array([[[[2.0, 4.0], [6.0, 10.0]], [[-1.0, -1.0], [-1.0, -1.0]]]])
    y = o.minmax_scale(x)
    assert np.array_equal(y[0, 0], np.array([[0.0, 0.25], [0.5, 1.0]]))
    assert np.array_equal(y[0, 1], np.zeros((2, 2)))
    g = np.random.default_rng(3)
    z = g.integers(-50, 50, size=(3, 2, 5, 5)).astype(np.float64)
    assert np.array_equal(o.minmax_scale(z), o.minmax_scale(4.0 * z + 8.0))   # exact: integer data, power-of-2 scale
    s = o.minmax_scale(z)
    for p in range(3):
        for c in range(2):
            assert s[p, c].min() == 0.0 and s[p, c].max() == 1.0
    assert o.minmax_scale(z.astype(np.float32)).dtype == np.float32


def test_augment_pins(oracle_mod):
    """Forward differences are exact on linear data and give 2j + 1 on j^2
    (h = 1); layout [s | D_x | D_y] with the stated sizes."""
    o = oracle_mod
    n = 5
    j = np.arange(n, dtype=np.float64)
    ramp_x = np.broadcast_to(j, (n, n))                     # s[i][j] = j
    ramp_y = ramp_x.T.copy()                                # s[i][j] = i
    a = o.augment(np.stack([ramp_x, ramp_y])[None], n, L=n - 1.0)
    ne = n * (n - 1)
    assert a.shape == (1, 2 * n * n + 4 * ne)
    dx, dy = a[0, 2 * n * n: 2 * n * n + 2 * ne], a[0, 2 * n * n + 2 * ne:]
    assert np.array_equal(dx[:ne], np.ones(ne)) and np.array_equal(dx[ne:], np.zeros(ne))
    assert np.array_equal(dy[:ne], np.zeros(ne)) and np.array_equal(dy[ne:], np.ones(ne))
    q = np.broadcast_to(j * j, (n, n))
    a = o.augment(np.stack([q, q])[None], n, L=n - 1.0)
    assert np.array_equal(a[0, 2 * n * n: 2 * n * n + n - 1], 2 * j[:-1] + 1)
    # h = L / (n - 1): doubling L halves the differences exactly
    a2 = o.augment(np.stack([q, q])[None], n, L=2 * (n - 1.0))
    assert np.array_equal(a2[0, 2 * n * n:], a[0, 2 * n * n:] / 2)


def test_w12_is_the_l2_distance_of_augmented_vectors(oracle_mod):
    """Eq. norm:W12: ||u||^2 + ||D_x u||^2 + ||D_y u||^2 computed part by part
    equals the squared L2 distance of the augmented vectors."""
    o = oracle_mod
    g = np.random.default_rng(4)
    n = 6
    A = g.standard_normal((3, 2, n, n))
    B = g.standard_normal((2, 2, n, n))
    Aa, Ba = o.augment(A, n, 1.0), o.augment(B, n, 1.0)
    D = o.pair_d2(Aa, Ba)
    h = 1.0 / (n - 1)
    for i in range(3):
        for k in range(2):
            u = A[i] - B[k]
            parts = (u ** 2).sum() + (((u[:, :, 1:] - u[:, :, :-1]) / h) ** 2).sum() + \
                (((u[:, 1:, :] - u[:, :-1, :]) / h) ** 2).sum()
            assert D[i, k] == pytest.approx(parts, rel=1e-12)


def test_pair_maxabs_brute_force(oracle_mod):
    """Eqs. norm:Linf / norm:W1inf / norm:W1infprime on tiny sets, against
    pure-Python loops; identical vectors give 0, one changed element gives
    its change; an empty segment gives 0."""
    o = oracle_mod
    g = np.random.default_rng(5)
    A = g.standard_normal((3, 11))
    B = g.standard_normal((4, 11))
    ends = [4, 4, 9, 11]
    D = o.pair_maxabs(A, B, ends)
    for i in range(3):
        for j in range(4):
            prev = 0
            for s, e in enumerate(ends):
                want = max((abs(float(A[i, k]) - float(B[j, k])) for k in range(prev, e)), default=0.0)
                assert D[i, j, s] == want
                prev = e
    C = A.copy()
    C[1, 7] += 0.5
    D2 = o.pair_maxabs(A, C, [11])
    assert D2[0, 0, 0] == 0.0 and D2[1, 1, 0] == abs((A[1, 7] + 0.5) - A[1, 7])
    W = o.combine_segments(D, 0)
    S = o.combine_segments(D, 1)
    R = o.combine_segments(D, 2)
    assert np.array_equal(W, np.max(D, axis=2))
    assert np.array_equal(S, ((D[..., 0] + D[..., 1]) + D[..., 2]) + D[..., 3])
    for i in range(3):
        for j in range(4):
            want = ((math.sqrt(D[i, j, 0]) + math.sqrt(D[i, j, 1])) + math.sqrt(D[i, j, 2])) + math.sqrt(D[i, j, 3])
            assert R[i, j] == want


def test_bins_from_values_brute_force(oracle_mod):
    o = oracle_mod
    g = np.random.default_rng(6)
    V = g.random(200)
    r = np.array([0.9, 0.5, 0.25, 0.1])
    V[:4] = r                                       # ties: strict, a value at R_m is not under it
    b = o.bins_from_values(V, r)
    for p in range(V.size):
        assert b[p] == sum(1 for m in range(r.size) if V[p] < r[m])
    c = o.counts_from_values(V, r)
    assert np.array_equal(c, np.array([(b >= m + 1).sum() for m in range(r.size)]))


def test_w12_sum_variant_from_part_distances(oracle_mod):
    """Eq. norm:W12prime: ||u|| + ||D_x u|| + ||D_y u|| equals the sum of the
    square roots of the per-part squared distances of augmented vectors."""
    o = oracle_mod
    g = np.random.default_rng(7)
    n = 5
    A = g.standard_normal((2, 2, n, n))
    B = g.standard_normal((3, 2, n, n))
    Aa, Ba = o.augment(A, n, 2.0), o.augment(B, n, 2.0)
    e = [2 * n * n, 2 * n * n + 2 * n * (n - 1), 2 * n * n + 4 * n * (n - 1)]
    parts = np.stack([o.pair_d2(Aa[:, a:b], Ba[:, a:b]) for a, b in zip([0] + e[:-1], e)], axis=-1)
    W = o.combine_segments(parts, 2)
    h = 2.0 / (n - 1)
    for i in range(2):
        for k in range(3):
            u = A[i] - B[k]
            want = np.sqrt((u ** 2).sum()) + np.sqrt((((u[:, :, 1:] - u[:, :, :-1]) / h) ** 2).sum()) + \
                np.sqrt((((u[:, 1:, :] - u[:, :-1, :]) / h) ** 2).sum())
            assert W[i, k] == pytest.approx(want, rel=1e-12)


# ---- second-order IMEX stepper (semi-implicit BDF2)

def _heat_modes(n, L, nu):
    h = L / (n - 1)
    i = np.arange(n)
    mode = lambda k: np.cos(np.pi * k * (i + 0.5) / n)
    lam = lambda k: (4.0 / h ** 2) * np.sin(np.pi * k / (2 * n)) ** 2
    shapes = [np.outer(mode(2), mode(3)), np.outer(mode(5), mode(1))]
    mu = np.array([nu[0] * (lam(2) + lam(3)), nu[1] * (lam(5) + lam(1))])
    return shapes, mu


@pytest.mark.parametrize("dt,S", [(1e-3, 1), (1e-3, 2), (1e-3, 50), (2e-2, 40)])
def test_sbdf2_heat_mode_closed_form(oracle_mod, dt, S):
    """Pure diffusion of one cosine mode per species (an eigenvector of the
    ghost-copy Laplacian, eigenvalue -mu/nu): the amplitude follows the linear
    recurrence a_1 = a_0 / (1 + dt mu), (3 + 2 dt mu) a_s = 4 a_{s-1} - a_{s-2},
    solved in closed form from the roots of its characteristic polynomial
    (complex for 2 dt mu > 1, the last case)."""
    n, L, nu = 16, 1.0, (0.3, 0.7)
    shapes, mu = _heat_modes(n, L, nu)
    a0 = np.array([1.0, 0.5])
    st = np.stack([a0[0] * shapes[0], a0[1] * shapes[1]])[None]
    out, steps, _, _ = oracle_mod.imex_run(oracle_mod.HEAT, (0.0, 0.0), nu, n, L, dt, S, state=st.copy(),
                                           scheme="sbdf2")
    c = 3.0 + 2.0 * dt * mu
    disc = np.sqrt((1.0 - 2.0 * dt * mu).astype(complex))
    zp, zm = (2.0 + disc) / c, (2.0 - disc) / c
    a1 = a0 / (1.0 + dt * mu)
    cp = (a1 - a0 * zm) / (zp - zm)
    a = (cp * zp ** S + (a0 - cp) * zm ** S).real
    want = np.stack([a[0] * shapes[0], a[1] * shapes[1]])
    assert steps[0] == S
    assert np.abs(out[0] - want).max() <= 1e-13


def test_sbdf2_is_second_order_against_the_exact_heat_solution(oracle_mod):
    """Error at T = 0.1 against exp(-mu t) of each mode: halving dt divides it
    by 4 for the second-order stepper and by 2 for IMEX Euler."""
    n, L, nu, T = 16, 1.0, (0.3, 0.7), 0.1
    shapes, mu = _heat_modes(n, L, nu)
    st = np.stack([shapes[0], 0.5 * shapes[1]])[None]
    a = np.array([1.0, 0.5]) * np.exp(-mu * T)
    want = np.stack([a[0] * shapes[0], a[1] * shapes[1]])
    for scheme, lo, hi in (("sbdf2", 3.7, 4.6), ("euler", 1.9, 2.1)):
        e = []
        for m in (20, 40, 80):
            out, _, _, _ = oracle_mod.imex_run(oracle_mod.HEAT, (0.0, 0.0), nu, n, L, T / m, m, state=st.copy(),
                                               scheme=scheme)
            e.append(np.abs(out[0] - want).max())
        assert lo < e[0] / e[1] < hi and lo < e[1] / e[2] < hi, (scheme, e)


def test_sbdf2_reaction_extrapolation_is_second_order(oracle_mod):
    """FitzHugh-Nagumo (nonlinear reaction) to T = 0.5: differences of runs
    at dt, dt/2, dt/4, dt/8 shrink 4-fold (2-fold for IMEX Euler), which a
    reaction taken at the old level only, or a wrong extrapolation weight,
    would not give."""
    n, L = 16, 1.0
    x = np.linspace(0.0, 1.0, n)
    ic = np.stack([0.1 * np.outer(np.cos(np.pi * x), np.cos(2 * np.pi * x)),
                   0.1 * np.outer(np.sin(np.pi * x), np.cos(np.pi * x))])[None]
    T = 0.5
    for scheme, lo, hi in (("sbdf2", 3.6, 4.4), ("euler", 1.8, 2.2)):
        us = [oracle_mod.imex_run(oracle_mod.FHN, (1.0, 10.0, 1.0), (0.05, 0.00028), n, L, T / m, m,
                                  state=ic.copy(), scheme=scheme)[0][0] for m in (50, 100, 200, 400)]
        e = [np.abs(us[j] - us[j + 1]).max() for j in range(3)]
        assert lo < e[0] / e[1] < hi and lo < e[1] / e[2] < hi, (scheme, e)


def test_sbdf2_keeps_a_stationary_state(oracle_mod):
    """A stationary state of the method-of-lines system is a fixed point of
    both steppers: started at IMEX Euler's converged Gierer-Meinhardt pattern
    (residual < 1e-11), 200 second-order steps move it by less than 1e-9."""
    w = cs.WORKLOADS["gm_source64_stationary"]
    n = 16
    base = oracle_mod.homogeneous_state(w["model"], w["params"])
    ic = cs.initial_conditions(base, n, 1, seed=5, law=w["ic_law"])
    L = w["L"] * n / w["n"]
    st, _, res, stat = oracle_mod.imex_run(w["model"], w["params"], w["nu"], n, L, w["dt"], 50000, 1e-11, 25,
                                           state=ic.copy())
    assert stat[0] == 0 and res[0] < 1e-11
    out, _, res2, _ = oracle_mod.imex_run(w["model"], w["params"], w["nu"], n, L, w["dt"], 200, state=st.copy(),
                                          scheme="sbdf2")
    assert np.abs(out - st).max() < 1e-9 and res2[0] < 1e-10
