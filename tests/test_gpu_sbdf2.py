"""GPU parity of the second-order IMEX stepper (semi-implicit BDF2,
`cil_simulate_patterns_sbdf2`; the fused line kernel at n = 32 and n = 64 in
FP32, the plain back-end elsewhere or on request) against the FP64 oracle.

Error measure and bars as for IMEX Euler: max |gpu - oracle| / max |oracle|;
1e-10 for FP64 at fixed step counts, 1e-4 for FP32; residual-stopped FP64
runs take the oracle's step counts.  A diffusing cosine mode is compared
with the closed-form solution of its recurrence.
"""
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


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("case,n,L,dt,steps", [(FHN, 32, 1.0, 0.01, 300), (GM, 17, 1.0, 0.05, 200),
                                               (GMS, 33, 60.0, 0.2, 150), (BZ, 64, 1.0, 0.05, 120),
                                               (FHN, 2, 1.0, 0.01, 50), (GMS, 32, 60.0, 0.2, 150),
                                               (BZ, 32, 1.0, 0.05, 200)])
def test_fp64_trajectory_parity(cil, oracle_mod, path, case, n, L, dt, steps):
    model, p, nu = case
    print("sbdf2 fp64 model=%d n=%d path=%d" % (model, n, path), flush=True)
    base = oracle_mod.homogeneous_state(model, p)
    ics = cs.initial_conditions(base, n, 3, seed=60 + model, law="additive_pos")
    st = torch.tensor(ics, dtype=torch.float64, device="cuda")
    rep = cil.cil_simulate_patterns(model, st, cil.make_problems(n, L, nu, p, count=3), dt, steps,
                                    check_every=steps, scheme="sbdf2", path=path)
    out, _, ores, _ = oracle_mod.imex_run(model, p, nu, n, L, dt, steps, 0.0, steps, state=ics.copy(), nthreads=8,
                                          scheme="sbdf2")
    assert rel_err(st.cpu().numpy(), out) <= 1e-10
    assert np.all(rep["steps_taken"] == steps) and np.all(rep["status"] == 0)
    assert np.allclose(rep["final_resid"], ores, rtol=1e-6, atol=1e-14)


def test_ragged_sides_and_offsets(cil, oracle_mod):
    """One call over sides 17, 32, 33 and 8 at explicit, gapped element
    offsets; each solve against its own oracle run."""
    model, p, nu = FHN
    sides = [17, 32, 33, 8]
    base = oracle_mod.homogeneous_state(model, p)
    ics = [cs.initial_conditions(base, n, 1, seed=70 + n, law="additive_sym")[0] for n in sides]
    offs, t = [], 0
    for n in sides:
        offs.append(t)
        t += 2 * n * n + 5                                   # a gap after every solve
    buf = np.full(t, 7.0)
    for o_, x in zip(offs, ics):
        buf[o_:o_ + x.size] = x.reshape(-1)
    st = torch.tensor(buf, device="cuda")
    probs = cil.make_problems(sides, 1.0, nu, p)
    cil.cil_simulate_patterns(model, st, probs, 0.01, 200, check_every=50, offsets=offs, scheme="sbdf2")
    g = st.cpu().numpy()
    for o_, x, n in zip(offs, ics, sides):
        want, _, _, _ = oracle_mod.imex_run(model, p, nu, n, 1.0, 0.01, 200, 0.0, 50, state=x[None].copy(),
                                            scheme="sbdf2")
        assert rel_err(g[o_:o_ + x.size], want.reshape(-1)) <= 1e-10
        assert np.all(g[o_ + x.size:o_ + x.size + 5] == 7.0)    # the gaps are untouched


@pytest.mark.parametrize("n,L", [(16, 30.0), (32, 60.0)])
def test_residual_stopped_runs_take_the_oracles_steps(cil, oracle_mod, n, L):
    model, p, nu = GMS
    dt, tol, check = 0.2, 1e-8, 25
    base = oracle_mod.homogeneous_state(model, p)
    ics = cs.initial_conditions(base, n, 4, seed=81, law="multiplicative")
    st = torch.tensor(ics, device="cuda")
    rep = cil.cil_simulate_patterns(model, st, cil.make_problems(n, L, nu, p, count=4), dt, 20000, tol=tol,
                                    check_every=check, scheme="sbdf2")
    out, osteps, ores, ostat = oracle_mod.imex_run(model, p, nu, n, L, dt, 20000, tol, check, state=ics.copy(),
                                                   nthreads=8, scheme="sbdf2")
    print("sbdf2 steps to 1e-8:", rep["steps_taken"], "oracle:", osteps)
    assert np.all(ostat == 0) and np.all(rep["status"] == 0)
    assert np.array_equal(rep["steps_taken"], osteps)
    assert np.all(rep["final_resid"] < tol)
    assert rel_err(st.cpu().numpy(), out) <= 1e-8


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("dt,S", [(1e-3, 1), (1e-3, 50), (2e-2, 40)])
def test_heat_mode_closed_form(cil, oracle_mod, dt, S, n):
    L, nu = 1.0, (0.3, 0.7)
    h = L / (n - 1)
    i = np.arange(n)
    mode = lambda k: np.cos(np.pi * k * (i + 0.5) / n)
    lam = lambda k: (4.0 / h ** 2) * np.sin(np.pi * k / (2 * n)) ** 2
    shapes = [np.outer(mode(2), mode(3)), np.outer(mode(5), mode(1))]
    mu = np.array([nu[0] * (lam(2) + lam(3)), nu[1] * (lam(5) + lam(1))])
    a0 = np.array([1.0, 0.5])
    st = torch.tensor(np.stack([a0[0] * shapes[0], a0[1] * shapes[1]])[None], device="cuda")
    cil.cil_simulate_patterns(oracle_mod.HEAT, st, cil.make_problems(n, L, nu, (0.0, 0.0), count=1), dt, S,
                              check_every=S, scheme="sbdf2")
    c = 3.0 + 2.0 * dt * mu
    disc = np.sqrt((1.0 - 2.0 * dt * mu).astype(complex))
    zp, zm = (2.0 + disc) / c, (2.0 - disc) / c
    cp = (a0 / (1.0 + dt * mu) - a0 * zm) / (zp - zm)
    a = (cp * zp ** S + (a0 - cp) * zm ** S).real
    want = np.stack([a[0] * shapes[0], a[1] * shapes[1]])
    assert np.abs(st.cpu().numpy()[0] - want).max() <= 1e-13


@pytest.mark.parametrize("n,path", [(32, 0), (32, 1), (64, 0)])
def test_fp32_trajectory(cil, oracle_mod, n, path):
    model, p, nu = FHN
    L, dt = 1.0, 0.01
    base = oracle_mod.homogeneous_state(model, p)
    ics = cs.initial_conditions(base, n, 3, seed=90, law="additive_sym").astype(np.float32).astype(np.float64)
    st = torch.tensor(ics, dtype=torch.float32, device="cuda")
    cil.cil_simulate_patterns(model, st, cil.make_problems(n, L, nu, p, count=3), dt, 200, check_every=200,
                              scheme="sbdf2", polish=0, path=path)
    out, _, _, _ = oracle_mod.imex_run(model, p, nu, n, L, dt, 200, 0.0, 200, state=ics.copy(), scheme="sbdf2")
    assert rel_err(st.double().cpu().numpy(), out) <= 1e-4


@pytest.mark.parametrize("n,L", [(16, 30.0), (32, 60.0)])
def test_fp32_floor_status(cil, oracle_mod, n, L):
    """FP32 cannot certify 1e-12: the solves stop at the FP32 floor."""
    model, p, nu = GMS
    base = oracle_mod.homogeneous_state(model, p)
    st = torch.tensor(cs.initial_conditions(base, n, 2, seed=91, law="multiplicative"), dtype=torch.float32,
                      device="cuda")
    rep = cil.cil_simulate_patterns(model, st, cil.make_problems(n, L, nu, p, count=2), 0.2, 20000, tol=1e-12,
                                    check_every=25, scheme="sbdf2", polish=0, fp32_floor_ulps=32)
    assert np.all(rep["status"] == cil.CIL_SOLVE_FP32_FLOOR)


def test_sbdf2_argument_errors(cil):
    model, p, nu = FHN
    st = torch.zeros(1, 2, 32, 32, dtype=torch.float32, device="cuda")
    probs = cil.make_problems(32, 1.0, nu, p, count=1)
    with pytest.raises(cil.CilError):                      # no quad-lane kernel for this scheme
        cil.cil_simulate_patterns(model, st, probs, 0.01, 10, path=cil.CIL_PATH_FUSED_QUAD, scheme="sbdf2")
    st17 = torch.zeros(1, 2, 17, 17, dtype=torch.float32, device="cuda")
    with pytest.raises(cil.CilError):                      # no fused kernel for this side
        cil.cil_simulate_patterns(model, st17, cil.make_problems(17, 1.0, nu, p, count=1), 0.01, 10,
                                  path=cil.CIL_PATH_FUSED, scheme="sbdf2")
    st64 = torch.zeros(1, 2, 64, 64, dtype=torch.float64, device="cuda")
    with pytest.raises(cil.CilError):                      # FP64 history at n = 64 does not fit the LDS
        cil.cil_simulate_patterns(model, st64, cil.make_problems(64, 1.0, nu, p, count=1), 0.01, 10,
                                  path=cil.CIL_PATH_FUSED_LINE, scheme="sbdf2")
    with pytest.raises(cil.CilError):                      # no FP64 polish
        cil.cil_simulate_patterns(model, st, probs, 0.01, 10, tol=1e-8, polish=1, scheme="sbdf2")
    with pytest.raises(ValueError):
        cil.cil_simulate_patterns(model, st, probs, 0.01, 10, scheme="rk4")
    rep = cil.cil_simulate_patterns(model, st, probs, 0.01, 0, scheme="sbdf2")
    assert rep["steps_taken"][0] == 0 and float(st.abs().max()) == 0.0
