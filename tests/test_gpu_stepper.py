"""GPU parity of the IMEX stepper against the FP64 oracle (through the C ABI).

Error measure for trajectories: max |gpu - oracle| / max |oracle| over the
whole state (FHN states sit near 0, so a pointwise relative error is
meaningless).  Bars: 1e-10 for FP64 at a fixed step count, 1e-4 for FP32 at
<= 500 steps (pattern selection amplifies rounding differences over longer
horizons).
"""
import math

import numpy as np
import pytest

import cil_synth as cs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FHN = (0, (1.0, 10.0, 1.0), (0.05, 0.00028))
GM = (1, (0.5, 1.0), (0.00025, 0.01))
GMS = (2, (0.5, 1.0), (1.0, 100.0))
BZ = (3, (4.5, 6.96), (0.0016, 0.0132))


@pytest.fixture(scope="module")
def cil():
    import paper_2203_14742_amd as c
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return c


def rel_err(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def run_both(cil, oracle_mod, model, p, nu, n, L, dt, steps, ics, prec, path, tol=0.0, check=None):
    B = ics.shape[0]
    check = check or steps
    probs = cil.make_problems(n, L, nu, p, count=B)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    st = torch.tensor(ics, dtype=dtype, device="cuda")
    rep = cil.cil_simulate_patterns(model, st, probs, dt, steps, tol=tol, check_every=check, path=path)
    torch.cuda.synchronize()
    out, osteps, ores, ostat = oracle_mod.imex_run(model, p, nu, n, L, dt, steps, tol, check,
                                                   state=ics.astype(np.float64), nthreads=8)
    return st.double().cpu().numpy(), rep, out, osteps, ores, ostat


@pytest.mark.parametrize("path", [1, 3, 4])
@pytest.mark.parametrize("case,n,L,dt,steps", [(FHN, 32, 1.0, 0.01, 300), (GM, 32, 1.0, 0.05, 200),
                                               (GMS, 64, 120.0, 0.2, 150), (BZ, 64, 1.0, 0.05, 200)])
def test_fp64_trajectory_parity(cil, oracle_mod, path, case, n, L, dt, steps):
    model, p, nu = case
    base = oracle_mod.homogeneous_state(model, p)
    print("fp64 parity model=%d n=%d path=%d" % (model, n, path), flush=True)
    ics = cs.initial_conditions(base, n, 3, seed=20 + model, law="additive_pos")
    g, rep, o, _, ores, _ = run_both(cil, oracle_mod, model, p, nu, n, L, dt, steps, ics, "fp64", path)
    assert rel_err(g, o) <= 1e-10
    assert np.all(rep["steps_taken"] == steps) and np.all(rep["status"] == 0)
    assert np.allclose(rep["final_resid"], ores, rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("path", [1, 3, 4])
@pytest.mark.parametrize("case,n,L,dt,steps", [(FHN, 32, 1.0, 0.01, 300), (GMS, 64, 120.0, 0.2, 150),
                                               (BZ, 128, 1.0, 0.05, 100), (FHN, 128, 1.0, 0.05, 100)])
def test_fp32_trajectory_parity(cil, oracle_mod, path, case, n, L, dt, steps):
    model, p, nu = case
    base = oracle_mod.homogeneous_state(model, p)
    print("fp32 parity model=%d n=%d path=%d" % (model, n, path), flush=True)
    ics = cs.initial_conditions(base, n, 2, seed=30 + model, law="additive_pos").astype(np.float32)
    g, rep, o, _, _, _ = run_both(cil, oracle_mod, model, p, nu, n, L, dt, steps,
                                  ics.astype(np.float64), "fp32", path)
    assert rel_err(g, o) <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,k,l", [(32, 3, 8), (64, 0, 5), (128, 17, 2), (20, 4, 4)])
def test_cosine_mode_decay_closed_form(cil, prec, n, k, l):
    """P2 on the GPU: a cosine mode decays by exactly (1 + dt nu Lambda_kl)^-s."""
    if prec == "fp64" and n == 128:
        path = 1
    else:
        path = 0
    L, dt, steps, nu = 1.0, 0.01, 40, (0.05, 0.002)
    mode = cs.cosine_mode(n, k, l)
    ics = np.stack([mode, -2.0 * mode])[None]
    dtype = torch.float64 if prec == "fp64" else torch.float32
    st = torch.tensor(ics, dtype=dtype, device="cuda")
    cil.cil_simulate_patterns(4, st, cil.make_problems(n, L, nu, (0.0,)), dt, steps, path=path)
    h = L / (n - 1)
    lam = (4 / h ** 2) * (math.sin(math.pi * k / (2 * n)) ** 2 + math.sin(math.pi * l / (2 * n)) ** 2)
    out = st.double().cpu().numpy()[0]
    # rounding accumulates per step: a few transforms of length n per step
    tol = (1e-14 if prec == "fp64" else 2e-7) * steps
    for s, sign in ((0, 1.0), (1, -2.0)):
        amp = (1 + dt * nu[s] * lam) ** (-steps)
        assert np.abs(out[s] - sign * amp * mode).max() <= tol * abs(sign)


@pytest.mark.parametrize("prec,path", [("fp64", 1), ("fp64", 3), ("fp64", 4), ("fp32", 3), ("fp32", 4)])
def test_homogeneous_state_stays_fixed(cil, oracle_mod, prec, path):
    model, p, nu = GMS
    v0, w0 = oracle_mod.homogeneous_state(model, p)
    n = 64
    ics = np.empty((2, 2, n, n))
    ics[:, 0] = v0
    ics[:, 1] = w0
    dtype = torch.float64 if prec == "fp64" else torch.float32
    st = torch.tensor(ics, dtype=dtype, device="cuda")
    cil.cil_simulate_patterns(model, st, cil.make_problems(n, 120.0, nu, p, count=2), 0.2, 50, path=path)
    out = st.double().cpu().numpy()
    # fixed up to rounding drift (dense length-64 cosine sums on the plain path)
    tol = 2e-12 if prec == "fp64" else 1e-6
    assert np.abs(out[:, 0] - v0).max() <= tol * v0 and np.abs(out[:, 1] - w0).max() <= tol * w0


@pytest.mark.parametrize("prec,path", [("fp64", 1), ("fp64", 3), ("fp64", 4), ("fp32", 1), ("fp32", 3),
                                       ("fp32", 4)])
def test_resume_is_bitwise(cil, prec, path):
    model, p, nu = FHN
    n = 32
    ics = cs.initial_conditions((0.0, 0.0), n, 3, seed=5, law="additive_sym")
    dtype = torch.float64 if prec == "fp64" else torch.float32
    probs = cil.make_problems(n, 1.0, nu, p, count=3)
    a = torch.tensor(ics, dtype=dtype, device="cuda")
    cil.cil_simulate_patterns(model, a, probs, 0.01, 70, check_every=70, path=path)
    b = torch.tensor(ics, dtype=dtype, device="cuda")
    cil.cil_simulate_patterns(model, b, probs, 0.01, 30, check_every=30, path=path)
    cil.cil_simulate_patterns(model, b, probs, 0.01, 40, check_every=40, path=path)
    assert torch.equal(a, b)


def test_check_every_does_not_change_the_trajectory(cil):
    model, p, nu = BZ
    n = 64
    ics = cs.initial_conditions((4.5, 6.96 / 4.5), n, 2, seed=9)
    probs = cil.make_problems(n, 1.0, nu, p, count=2)
    a = torch.tensor(ics, dtype=torch.float32, device="cuda")
    cil.cil_simulate_patterns(model, a, probs, 0.05, 60, check_every=60)
    b = torch.tensor(ics, dtype=torch.float32, device="cuda")
    cil.cil_simulate_patterns(model, b, probs, 0.05, 60, check_every=7)
    assert torch.equal(a, b)


@pytest.mark.parametrize("path", [1, 3, 4])
def test_stop_rule_matches_oracle(cil, oracle_mod, path):
    """tol > 0: a solve stops at the first multiple of check_every whose FP64
    residual is below tol; FP64 steps_taken equal the oracle's."""
    model, p, nu = GMS
    n, L, dt = 32, 60.0, 0.2
    base = oracle_mod.homogeneous_state(model, p)
    ics = cs.initial_conditions(base, n, 4, seed=41, law="multiplicative")
    tol, check = 1e-7, 10
    g, rep, o, osteps, ores, ostat = run_both(cil, oracle_mod, model, p, nu, n, L, dt, 5000, ics, "fp64", path,
                                              tol=tol, check=check)
    assert np.all(ostat == 0) and np.all(rep["status"] == 0)
    # steps agree unless the oracle residual sits within rounding of tol at a check
    assert np.array_equal(rep["steps_taken"], osteps)
    assert np.all(rep["final_resid"] < tol)
    assert rel_err(g, o) <= 1e-9


def gms_mol_rhs(u, p, nu, n, L):
    """nu Lap_h u + F(u) of the GM-source model for states u [S, 2, n, n]:
    five-point Laplacian with ghost copies of the edge values (test-local
    arithmetic, so that no GPU result goes into the oracle)."""
    h = L / (n - 1)
    q = np.pad(u, ((0, 0), (0, 0), (1, 1), (1, 1)), mode="edge")
    lap = (q[:, :, :-2, 1:-1] + q[:, :, 2:, 1:-1] + q[:, :, 1:-1, :-2] + q[:, :, 1:-1, 2:] - 4.0 * u) / (h * h)
    v, z = u[:, 0], u[:, 1]
    a, b = p[0], p[1]
    return np.stack([nu[0] * lap[:, 0] + a - b * v + v * v / z, nu[1] * lap[:, 1] + v * v - z], axis=1)


def test_gms_mol_rhs_against_the_oracle(oracle_mod):
    """The test-local right-hand side above equals the oracle's on random states."""
    model, p, nu = GMS
    u = 1.0 + np.random.default_rng(4).random((2, 2, 9, 9))
    want = np.stack([oracle_mod.mol_rhs(model, p, nu, 9, 7.0, u[b]) for b in range(2)])
    assert np.abs(gms_mol_rhs(u, p, nu, 9, 7.0) - want).max() <= 1e-12 * np.abs(want).max()


def test_fp32_polish_reaches_fp64_tolerance(cil, oracle_mod):
    """FP32 stepping stalls at its floor; the polish phase continues in FP64 on
    the GPU until the 1e-8 residual is met; the returned pattern is a
    stationary solution of the stencil system to FP32 rounding."""
    model, p, nu = GMS
    n, L, dt = 64, 120.0, 0.2
    base = oracle_mod.homogeneous_state(model, p)
    ics = cs.initial_conditions(base, n, 4, seed=3, law="multiplicative")
    st = torch.tensor(ics, dtype=torch.float32, device="cuda")
    rep = cil.cil_simulate_patterns(model, st, cil.make_problems(n, L, nu, p, count=4), dt, 20000, tol=1e-8,
                                    check_every=25)
    assert np.all(rep["status"] == 0), rep
    assert np.all(rep["final_resid"] < 1e-8)
    assert np.all(rep["steps_fp64"] > 0) and np.all(rep["steps_fp64"] < rep["steps_taken"])
    out = st.double().cpu().numpy()
    assert np.abs(gms_mol_rhs(out, p, nu, n, L)).max() < 1e-4    # fp32 rounding of a stationary state
    # without polish: FP32 floor status
    st2 = torch.tensor(ics, dtype=torch.float32, device="cuda")
    rep2 = cil.cil_simulate_patterns(model, st2, cil.make_problems(n, L, nu, p, count=4), dt, 20000, tol=1e-8,
                                     check_every=25, polish=0)
    assert np.all(rep2["status"] == cil.CIL_SOLVE_FP32_FLOOR)


def test_uneven_batch_matches_oracle(cil, oracle_mod):
    """Solves of different grid sides and parameters in one call."""
    model, p0, nu0 = BZ
    ns = [32, 64, 17, 128, 32]
    params = cs.relative_draws(p0, len(ns), 0.05, seed=4)
    nus = cs.relative_draws(nu0, len(ns), 0.05, seed=5)
    ics = []
    for b, n in enumerate(ns):
        base = oracle_mod.homogeneous_state(model, params[b])
        ics.append(cs.initial_conditions(base, n, 1, seed=50 + b)[0])
    flat = np.concatenate([x.reshape(-1) for x in ics])
    probs = cil.make_problems(ns, 1.0, nus, params)
    st = torch.tensor(flat, dtype=torch.float64, device="cuda")
    rep = cil.cil_simulate_patterns(model, st, probs, 0.05, 120, check_every=40)
    outs, osteps, _, _ = oracle_mod.imex_run(model, params, nus, ns, 1.0, 0.05, 120, 0.0, 40, state=ics)
    g = st.cpu().numpy()
    off = 0
    for b, n in enumerate(ns):
        gb = g[off: off + 2 * n * n].reshape(2, n, n)
        off += 2 * n * n
        assert rel_err(gb, outs[b]) <= 1e-10, (b, n)
    assert np.all(rep["steps_taken"] == 120)


def test_nonfinite_solve_is_reported(cil):
    model, p, nu = GMS
    n = 32
    ics = cs.initial_conditions((1.5, 2.25), n, 3, seed=1, law="multiplicative")
    ics[1, 1, 5, 5] = np.nan
    st = torch.tensor(ics, dtype=torch.float32, device="cuda")
    rep = cil.cil_simulate_patterns(model, st, cil.make_problems(n, 60.0, nu, p, count=3), 0.2, 20,
                                    check_every=10, raise_on_nonfinite=False)
    assert list(rep["status"]) == [0, cil.CIL_SOLVE_NONFINITE, 0]
    assert rep["steps_taken"][1] == 10 and np.isnan(rep["final_resid"][1])
    with pytest.raises(cil.CilError) as e:
        st = torch.tensor(ics, dtype=torch.float32, device="cuda")
        cil.cil_simulate_patterns(model, st, cil.make_problems(n, 60.0, nu, p, count=3), 0.2, 20, check_every=10)
    assert e.value.code == cil.CIL_ENONFINITE


def test_fused_unsupported_size_is_an_error(cil):
    st = torch.zeros((1, 2, 20, 20), dtype=torch.float64, device="cuda")
    with pytest.raises(cil.CilError) as e:
        cil.cil_simulate_patterns(0, st, cil.make_problems(20, 1.0, (0.1, 0.1), (1, 1, 1)), 0.01, 5, path=2)
    assert e.value.code == cil.CIL_EUNSUPPORTED


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("prec,case,n,L,dt,steps", [("fp64", FHN, 32, 1.0, 0.01, 200), ("fp64", GMS, 64, 120.0, 0.2, 150),
                                                    ("fp32", FHN, 32, 1.0, 0.01, 200), ("fp32", GMS, 64, 120.0, 0.2, 150),
                                                    ("fp32", BZ, 128, 1.0, 0.05, 60)])
def test_every_quad_shape_matches_oracle(cil, oracle_mod, shape, prec, case, n, L, dt, steps):
    """Each code shape of the fused quad-lane stepper takes the same steps:
    trajectory parity and the stop rule (resid checked every 25 steps)."""
    model, p, nu = case
    base = oracle_mod.homogeneous_state(model, p)
    print("quad shape %d %s model=%d n=%d" % (shape, prec, model, n), flush=True)
    ics = cs.initial_conditions(base, n, 3, seed=40 + model, law="additive_pos")
    if prec == "fp32":
        ics = ics.astype(np.float32).astype(np.float64)
    cil.cil_set_option(cil.CIL_OPT_QUAD_SHAPE, shape)
    try:
        g, rep, o, osteps, ores, ostat = run_both(cil, oracle_mod, model, p, nu, n, L, dt, steps, ics, prec, 4,
                                                  check=25)
    finally:
        cil.cil_set_option(cil.CIL_OPT_QUAD_SHAPE, -1)
    assert rel_err(g, o) <= (1e-10 if prec == "fp64" else 1e-4)
    assert np.array_equal(rep["steps_taken"], osteps)
    if prec == "fp64":
        assert np.allclose(rep["final_resid"], ores, rtol=1e-6, atol=1e-14)


def test_quad_shape_option_range(cil):
    with pytest.raises(cil.CilError) as e:
        cil.cil_set_option(cil.CIL_OPT_QUAD_SHAPE, 4)
    assert e.value.code == cil.CIL_EINVAL


def test_wave_priority_changes_timing_only(cil):
    """Residual-driven issue priority: identical states, steps and residuals
    with it on (default) and off."""
    w = cs.WORKLOADS["gm_source64_stationary"]
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics = cs.initial_conditions(base, w["n"], 40, seed=41, law=w["ic_law"])
    probs = cil.make_problems(w["n"], w["L"], w["nu"], w["params"], count=40)
    out = []
    try:
        for prio in (0, 100):
            cil.cil_set_option(cil.CIL_OPT_WAVE_PRIORITY, prio)
            st = torch.tensor(ics, dtype=torch.float64, device="cuda")
            rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                            check_every=w["check_every"])
            out.append((st, rep))
    finally:
        cil.cil_set_option(cil.CIL_OPT_WAVE_PRIORITY, 100)
    assert torch.equal(out[0][0], out[1][0])
    for k in ("steps_taken", "final_resid", "status"):
        assert np.array_equal(out[0][1][k], out[1][1][k])
    assert np.all(out[1][1]["status"] == 0)
    for bad in (1, -1, 2000000):
        with pytest.raises(cil.CilError):
            cil.cil_set_option(cil.CIL_OPT_WAVE_PRIORITY, bad)


def test_polling_waits_change_nothing(cil, oracle_mod):
    """Host waits that poll (CIL_OPT_SYNC_SPIN_US, default) or block at once
    (0): the same stepping reports and the same adaptive bins and counts."""
    w = cs.WORKLOADS["gm_source64_stationary"]
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics = cs.initial_conditions(base, w["n"], 24, seed=43, law=w["ic_law"])
    probs = cil.make_problems(w["n"], w["L"], w["nu"], w["params"], count=24)
    out = []
    try:
        for spin in (0, 200000):
            cil.cil_set_option(cil.CIL_OPT_SYNC_SPIN_US, spin)
            st = torch.tensor(ics, dtype=torch.float32, device="cuda")
            rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                            check_every=w["check_every"], polish=2)
            P = st.reshape(24, -1)
            lo, hi, radii, bins, counts = cil.cil_pair_bins_adaptive(P[:12], P[12:], 8)
            out.append((st, rep, (lo, hi), bins, counts))
    finally:
        cil.cil_set_option(cil.CIL_OPT_SYNC_SPIN_US, 200000)
    (a, ra, ga, ba, ca), (b, rb, gb, bb, cb) = out
    assert torch.equal(a, b) and torch.equal(ba, bb) and ga == gb and np.array_equal(ca, cb)
    for k in ("steps_taken", "steps_fp64", "final_resid", "status"):
        assert np.array_equal(ra[k], rb[k]), k


def _gm_batch(cil, n, count, seed, L):
    w = cs.WORKLOADS["gm_source64_stationary"]
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics = cs.initial_conditions(base, n, count, seed=seed, law=w["ic_law"])
    return w, ics, cil.make_problems(n, L, w["nu"], w["params"], count=count)


@pytest.mark.parametrize("n,L", [(64, 120.0), (32, 60.0)])
def test_mixed_polish_equals_separate_launch(cil, n, L):
    """FP32 stepping with the FP64 polish inside one persistent launch gives
    the bits of the same kernel run as two launches (the FP32 phase of the
    whole batch, then the polish of the solves at their FP32 floor): states,
    step counts (total and FP64), residuals and statuses."""
    w, ics, probs = _gm_batch(cil, n, 24, seed=51 + n, L=L)
    out = []
    try:
        for sep in (0, 1):
            cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, sep)
            st = torch.tensor(ics, dtype=torch.float32, device="cuda")
            print("polish separate=%d n=%d" % (sep, n), flush=True)
            rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                            check_every=w["check_every"], polish=1)
            out.append((st, rep))
    finally:
        cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, 0)
    assert torch.equal(out[0][0], out[1][0])
    for k in ("steps_taken", "steps_fp64", "final_resid", "status"):
        assert np.array_equal(out[0][1][k], out[1][1][k]), k
    assert np.any(out[0][1]["steps_fp64"] > 0)            # solves reached the FP32 floor and were polished
    if n == 64:                                           # the benchmarked model and grid: all converge
        assert np.all(out[0][1]["steps_fp64"] > 0)
        assert np.all(out[0][1]["status"] == 0) and np.all(out[0][1]["final_resid"] < w["tol"])


@pytest.mark.parametrize("n,L", [(64, 120.0), (32, 60.0)])
def test_refinement_polish(cil, n, L):
    """The refinement polish (polish = 2: FP64 state, FP32 correction steps
    with the FP64 residual of the five-point system) gives the same bits
    inside the mixed launch and as a launch of its own; it stops where the
    FP64-step polish stops (same statuses, step counts within one
    evaluation interval) and its patterns agree with that polish's to two
    FP32 roundings plus the motion of one interval at the tolerance."""
    w, ics, probs = _gm_batch(cil, n, 24, seed=51 + n, L=L)
    out = []
    try:
        for polish, sep in ((2, 0), (2, 1), (1, 0)):
            cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, sep)
            st = torch.tensor(ics, dtype=torch.float32, device="cuda")
            print("polish=%d separate=%d n=%d" % (polish, sep, n), flush=True)
            rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                            check_every=w["check_every"], polish=polish)
            out.append((st, rep))
    finally:
        cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, 0)
    (a, ra), (b, rb), (c, rc) = out
    assert torch.equal(a, b)
    for k in ("steps_taken", "steps_fp64", "final_resid", "status"):
        assert np.array_equal(ra[k], rb[k]), k
    assert np.any(ra["steps_fp64"] > 0)
    assert np.array_equal(ra["status"], rc["status"])
    ok = ra["status"] == 0
    if n == 64:
        assert np.all(ok)
    assert np.all(ra["final_resid"][ok] < w["tol"])
    assert np.all(np.abs(ra["steps_taken"] - rc["steps_taken"]) <= w["check_every"])
    ga, gc = a.double().cpu().numpy(), c.double().cpu().numpy()
    diff = np.abs(ga - gc).reshape(len(probs), -1).max(axis=1)
    bar = 2.0 ** -22 * np.abs(gc).reshape(len(probs), -1).max(axis=1) + w["check_every"] * w["tol"] * w["dt"]
    print("refinement vs FP64-step polish: max difference %.3e (bar %.3e)" % (diff.max(), bar.min()))
    assert np.all(diff[ok] <= bar[ok])


@pytest.mark.parametrize("case,n,L,dt", [(FHN, 32, 1.0, 0.01), (GM, 32, 1.0, 0.05), (BZ, 32, 1.0, 0.05),
                                         (GMS, 32, 60.0, 0.2), (FHN, 64, 1.0, 0.01), (GM, 64, 1.0, 0.05),
                                         (BZ, 64, 1.0, 0.05), (GMS, 64, 120.0, 0.2)])
def test_refinement_form_every_model(cil, case, n, L, dt):
    """The refinement form's reaction change (kinetics_delta, per model) and
    its FP64 residual, against the FP64-step polish over 200 steps of each
    model's transient: a floor of 2^20 FP32 units switches every solve at its
    first evaluation (step 25), so both polishes run steps 25-225 from the
    same FP32 state.  They agree to FP32 rounding of the motion since the
    switch (measured up to 1.7e-5 of max|u|, GM source); a wrong or dropped
    term in the change of the reaction would put them apart by a fair part of
    that motion (over 1e-2)."""
    model, p, nu = case
    base = cil.cil_homogeneous_state(model, p)
    ics = cs.initial_conditions(base, n, 8, seed=80 + model, law="additive_pos")
    probs = cil.make_problems(n, L, nu, p, count=8)
    out = {}
    for polish in (1, 2):
        st = torch.tensor(ics, dtype=torch.float32, device="cuda")
        print("refinement model=%d n=%d polish=%d" % (model, n, polish), flush=True)
        rep = cil.cil_simulate_patterns(model, st, probs, dt, 225, tol=1e-8, check_every=25, polish=polish,
                                        fp32_floor_ulps=1 << 20)
        out[polish] = (st.double().cpu().numpy().reshape(8, -1), rep)
    (a, ra), (b, rb) = out[1], out[2]
    for r in (ra, rb):
        assert np.all(r["steps_fp64"] == 200) and np.all(r["steps_taken"] == 225)
        assert np.all(r["status"] == cil.CIL_SOLVE_MAXSTEPS)
    d = (np.abs(a - b).max(axis=1) / np.abs(a).max(axis=1)).max()
    print("refinement vs FP64-step polish after 200 steps: %.2e of max|u|" % d)
    assert d <= 1e-4


def test_mixed_polish_uneven_sides(cil):
    """Sides 32, 64 (mixed launches) and 128 (FP32 launch + FP64 polish in a
    launch of its own) in one call: identical to the separate polish
    launches."""
    w = cs.WORKLOADS["gm_source64_stationary"]
    ns = [32, 64, 128, 64, 32]
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    flat = np.concatenate([cs.initial_conditions(base, n, 1, seed=60 + i, law=w["ic_law"]).reshape(-1)
                           for i, n in enumerate(ns)])
    probs = cil.make_problems(ns, [60.0 if n == 32 else (120.0 if n == 64 else 240.0) for n in ns], w["nu"],
                              w["params"])
    out = []
    try:
        for sep in (0, 1):
            cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, sep)
            st = torch.tensor(flat, dtype=torch.float32, device="cuda")
            rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], 4000, tol=w["tol"],
                                            check_every=w["check_every"], polish=1)
            out.append((st, rep))
    finally:
        cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, 0)
    assert torch.equal(out[0][0], out[1][0])
    for k in ("steps_taken", "steps_fp64", "final_resid", "status"):
        assert np.array_equal(out[0][1][k], out[1][1][k]), k
