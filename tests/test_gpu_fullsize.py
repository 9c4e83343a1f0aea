"""Full-size parity of the benchmarked step (the launch configuration bench.py
times): 500 Gierer-Meinhardt (source form) solves on 64x64 grids to FP64
residual < 1e-8, then the CIL statistic of the two 250-pattern halves stored
as FP32 (d = 8192, 13 radii, 200 bootstrap resamples) and the likelihood.

The benchmarked stepping is FP32 with each solve's polish (from its FP32
floor to the tolerance) in the same launch, in the refinement form (FP64
state, FP32 correction steps); the FP64-step polish is checked the same way.
Their patterns are checked by properties that hold one by one: every stored
pattern is stationary under one IMEX-Euler step (residual within what FP32
storage rounding allows, tol + 4 x 2^-24 max|u| / dt; the step is evaluated
here with scipy's orthonormal DCT-II, itself checked on the oracle's
stationary patterns), and the whole batch is bit-identical to the same
kernel run as two launches (FP32 phase, then the polish).  The FP64 fused stepping is checked against the oracle directly
(sampled solves: step counts identical, patterns within 1e-8).  The
statistic is checked in full on the oracle's own 500 stationary patterns,
stored as FP32 and as FP64: the oracle computes all 62 500 canonical
distances, and range, radii, bins, counts, bootstrap counts (bit-exact) and
the likelihood (1e-10) must agree.
"""
import numpy as np
import pytest
from scipy.fft import dctn, idctn

import cil_synth as cs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cil():
    import paper_2203_14742_amd as c
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return c


@pytest.fixture(scope="module")
def stepped(cil):
    w = cs.WORKLOADS["gm_source64_stationary"]
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics = cs.initial_conditions(base, w["n"], w["count"], seed=w["seeds"][0], law=w["ic_law"])
    st = torch.tensor(ics, dtype=torch.float64, device="cuda")
    probs = cil.make_problems(w["n"], w["L"], w["nu"], w["params"], count=w["count"])
    print("full-size GM-source run", flush=True)
    rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                    check_every=w["check_every"], path=cil.CIL_PATH_AUTO)
    return w, ics, st, rep


@pytest.fixture(scope="module")
def oracle_stationary(oracle_mod):
    """All 500 solves run to the tolerance by the oracle (about 12 s on 16 threads)."""
    w = cs.WORKLOADS["gm_source64_stationary"]
    base = oracle_mod.homogeneous_state(w["model"], w["params"])
    ics = cs.initial_conditions(base, w["n"], w["count"], seed=w["seeds"][0], law=w["ic_law"])
    print("oracle: %d GM-source solves to stationarity" % w["count"], flush=True)
    out, steps, res, stat = oracle_mod.imex_run(w["model"], w["params"], w["nu"], w["n"], w["L"], w["dt"],
                                                w["max_steps"], w["tol"], w["check_every"], state=ics.copy(),
                                                nthreads=16)
    assert np.all(stat == 0)
    return out, res


def one_step_residual(u, w):
    """max |u' - u| / dt of one IMEX-Euler step of the GM-source model (a, b)
    from each state u [S, 2, n, n]: reaction u + dt F(u), then the diffusion
    solve in the orthonormal DCT-II basis, which diagonalises the ghost-copy
    Laplacian with eigenvalues -(4/h^2)(sin^2(pi k/2n) + sin^2(pi l/2n))."""
    n, L, dt, (a, b), nu = w["n"], w["L"], w["dt"], w["params"], w["nu"]
    h = L / (n - 1)
    s2 = np.sin(np.pi * np.arange(n) / (2 * n)) ** 2
    lam = (4.0 / h ** 2) * (s2[:, None] + s2[None, :])
    v, z = u[:, 0], u[:, 1]
    r = np.stack([v + dt * (a - b * v + v * v / z), z + dt * (v * v - z)], axis=1)
    out = np.empty_like(r)
    for sp in range(2):
        out[:, sp] = idctn(dctn(r[:, sp], type=2, norm="ortho", axes=(1, 2)) / (1.0 + dt * nu[sp] * lam),
                           type=2, norm="ortho", axes=(1, 2))
    return np.abs(out - u).reshape(u.shape[0], -1).max(axis=1) / dt


@pytest.fixture(scope="module")
def stepped32(cil):
    w = cs.WORKLOADS["gm_source64_stationary"]
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics = cs.initial_conditions(base, w["n"], w["count"], seed=w["seeds"][0], law=w["ic_law"])
    probs = cil.make_problems(w["n"], w["L"], w["nu"], w["params"], count=w["count"])
    out = {}
    try:
        for polish in (1, 2):
            for sep in (0, 1):
                cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, sep)
                st = torch.tensor(ics, dtype=torch.float32, device="cuda")
                print("full-size GM-source run, FP32 + polish %d (separate launch: %d)" % (polish, sep), flush=True)
                rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                                check_every=w["check_every"], polish=polish)
                out.setdefault(polish, []).append((st, rep))
    finally:
        cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, 0)
    return w, ics, out


@pytest.mark.parametrize("polish", [1, 2])
def test_full_workload_fp32_polished_patterns(cil, oracle_mod, stepped32, polish):
    """polish 1: FP64 steps from the FP32 floor; 2: the refinement form (FP64
    state, FP32 correction steps), the benchmarked configuration."""
    w, ics, out = stepped32
    (st, rep), (st2, rep2) = out[polish]
    assert torch.equal(st, st2)
    for k in ("steps_taken", "steps_fp64", "final_resid", "status"):
        assert np.array_equal(rep[k], rep2[k]), k
    assert np.all(rep["status"] == 0) and np.all(rep["final_resid"] < w["tol"])
    assert np.all(rep["steps_fp64"] > 0)
    g = st.double().cpu().numpy()
    r = one_step_residual(g, w)
    # FP32 storage moves each value by at most 2^-24 max|u|; one step maps that
    # perturbation to a residual of about that over dt (the diffusion solve
    # damps it, the explicit reaction adds dt |f'|); a factor 4 of margin
    bar = w["tol"] + 4.0 * 2.0 ** -24 * np.abs(g).reshape(g.shape[0], -1).max(axis=1) / w["dt"]
    print("FP32-stored polished patterns: one-step residual max %.3e (bar %.3e)" % (r.max(), bar.min()))
    assert np.all(r < bar)


def test_one_step_residual_on_the_oracles_patterns(oracle_stationary):
    """The residual function above against the oracle's own stopping residual
    on its stationary patterns (same definition, different arithmetic)."""
    w = cs.WORKLOADS["gm_source64_stationary"]
    out, res = oracle_stationary
    r = one_step_residual(out[:40], w)
    # one step beyond the oracle's stop: the residual decays, and the two
    # diffusion solvers differ by rounding only
    assert np.all(r < w["tol"]) and np.all(r <= res[:40] * 1.01 + 1e-12)


def test_full_workload_stationary_patterns(cil, oracle_mod, stepped):
    w, ics, st, rep = stepped
    assert np.all(rep["status"] == 0) and np.all(rep["final_resid"] < w["tol"])
    s = rep["steps_taken"]
    sample = sorted({int(np.argmax(s)), int(np.argmin(s)), 0, 123, 249, 250, 377, 499})
    out, osteps, ores, ostat = oracle_mod.imex_run(w["model"], w["params"], w["nu"], w["n"], w["L"], w["dt"],
                                                   w["max_steps"], w["tol"], w["check_every"],
                                                   state=ics[sample].copy(), nthreads=8)
    assert np.all(ostat == 0)
    assert np.array_equal(s[sample], osteps)
    g = st.cpu().numpy()[sample]
    err = np.abs(g - out).max() / np.abs(out).max()
    print("sampled stationary patterns: rel err %.3e, steps %s" % (err, list(osteps)))
    assert err <= 1e-8


@pytest.mark.parametrize("store", [np.float32, np.float64])
def test_full_workload_statistic(cil, oracle_mod, oracle_stationary, store):
    w = cs.WORKLOADS["gm_source64_stationary"]
    B, half, d, M = w["count"], w["count"] // 2, 2 * w["n"] ** 2, w["M"]
    Pn = oracle_stationary[0].reshape(B, d).astype(store)
    An, Bn = Pn[:half], Pn[half:]
    A, Bs = torch.from_numpy(An).cuda(), torch.from_numpy(Bn).cuda()
    D = oracle_mod.pair_d2(An, Bn, nthreads=8)
    lo, hi, radii, bins, counts = cil.cil_pair_bins_adaptive(A, Bs, M)     # as the benchmark runs it
    assert (lo, hi) == (D.min(), D.max())
    assert np.array_equal(radii, oracle_mod.radii_ladder(D.min(), D.max(), M))
    assert np.array_equal(bins.cpu().numpy(), oracle_mod.bins_from_d2(D, radii))
    assert np.array_equal(counts, oracle_mod.counts_from_d2(D, radii))
    assert cil.cil_distance_range(A, Bs) == (lo, hi)
    bins2, counts2 = cil.cil_pair_bins(A, Bs, cil.cil_radii(lo, hi, M))
    assert torch.equal(bins2, bins) and np.array_equal(counts2, counts)
    ia, ib = cs.resample_halves(half, half, half, half, w["n_boot"], seed=6)
    Yc, Y = cil.cil_bootstrap_features(bins, torch.from_numpy(ia), torch.from_numpy(ib), M)
    want_c, want_y = oracle_mod.bootstrap_vectors(D, ia, ib, radii, nthreads=8)
    assert np.array_equal(Yc.cpu().numpy(), want_c)
    assert np.array_equal(Y.cpu().numpy(), want_y)
    y_obs = oracle_mod.counts_from_d2(D, radii) / float(half * half)
    f, ll, me, stt = cil.cil_gaussian_loglik(Y, torch.tensor(y_obs, dtype=torch.float64, device="cuda"))
    r = oracle_mod.gaussian_cost(want_y, y_obs)
    assert int(me.cpu()[0]) == r["m_eff"]
    if r["ok"]:
        assert int(stt.cpu()[0]) == 0
        assert float(f.cpu()[0]) == pytest.approx(r["f"], rel=1e-10)
        assert float(ll.cpu()[0]) == pytest.approx(r["loglik"], rel=1e-10)
    else:
        assert int(stt.cpu()[0]) == cil.CIL_ENOTSPD
    print("full statistic: counts", counts.tolist(), "m_eff", r["m_eff"], "f", r.get("f"))
