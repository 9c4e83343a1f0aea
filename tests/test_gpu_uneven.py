"""Uneven batches: Brusselator solves of sides 32, 64 and 128 in one call, each
with its own (A, B, Du, Dv) drawn around Table exp1's point and accepted only
if Turing-unstable on its own grid.  The fused kernels of the three sides run
side by side on streams forked from the caller's stream.

Small batches are compared with the oracle solve by solve; the full batch of
the uneven workload (2048 solves, 2000 FP32 steps) is checked through its
reports and, for sampled solves, against the oracle over the first 300 steps
(beyond that, pattern selection amplifies FP32 rounding; the 1e-4 FP32 bar is
taken at <= 500 steps).
"""
import numpy as np
import pytest

import cil_synth as cs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cil():
    import paper_2203_14742_amd as c
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return c


def split(flat, ns):
    out, off = [], 0
    for n in ns:
        out.append(flat[off: off + 2 * n * n].reshape(2, n, n))
        off += 2 * n * n
    return out


def rel_err(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def problem(oracle_mod, count, seed, sides=(32, 64, 128)):
    ns, ps, nus = cs.brusselator_uneven(count, seed, sides=sides)
    bases = [oracle_mod.homogeneous_state(cs.BRUSSELATOR, p) for p in ps]
    flat = cs.uneven_initial_states(bases, ns, seed=seed + 100)
    return ns, ps, nus, flat


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_uneven_turing_batch_matches_oracle(cil, oracle_mod, prec):
    ns, ps, nus, flat = problem(oracle_mod, 9, seed=12)
    if prec == "fp32":
        flat = flat.astype(np.float32).astype(np.float64)
    dtype = torch.float32 if prec == "fp32" else torch.float64
    st = torch.tensor(flat, dtype=dtype, device="cuda")
    print("uneven %s sides %s" % (prec, ns), flush=True)
    rep = cil.cil_simulate_patterns(cs.BRUSSELATOR, st, cil.make_problems(ns, 1.0, nus, ps), 0.05, 150,
                                    check_every=50)
    outs, osteps, _, ostat = oracle_mod.imex_run(cs.BRUSSELATOR, ps, nus, ns, 1.0, 0.05, 150, 0.0, 50,
                                                 state=split(flat, ns), nthreads=8)
    g = split(st.double().cpu().numpy(), ns)
    bar = 1e-4 if prec == "fp32" else 1e-10
    for b, n in enumerate(ns):
        assert rel_err(g[b], outs[b]) <= bar, (b, n)
    assert np.all(rep["steps_taken"] == 150) and np.all(rep["status"] == 0)


def test_uneven_full_workload(cil, oracle_mod):
    w = cs.WORKLOADS["bz_uneven2048"]
    ns, ps, nus = cs.brusselator_uneven(w["count"], w["seed"], sides=w["sides"], rel=w["rel"])
    bases = [oracle_mod.homogeneous_state(w["model"], p) for p in ps]
    flat = cs.uneven_initial_states(bases, ns, seed=w["ic_seed"])
    probs = cil.make_problems(ns, w["L"], nus, ps)
    st = torch.tensor(flat, dtype=torch.float32, device="cuda")
    print("uneven full workload: %d solves" % len(ns), flush=True)
    rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], check_every=w["check_every"])
    assert np.all(rep["status"] == 0) and np.all(rep["steps_taken"] == w["max_steps"])
    assert torch.isfinite(st).all()
    # sampled solves, every side, against the oracle over 300 steps
    sample = [0, 1, 2, 1000, 1001, 1002, 2045, 2046, 2047]
    sub_ns = [ns[b] for b in sample]
    sub = [flat[sum(2 * m * m for m in ns[:b]):][:2 * ns[b] ** 2].astype(np.float32).astype(np.float64) for b in sample]
    sflat = np.concatenate(sub)
    st2 = torch.tensor(sflat, dtype=torch.float32, device="cuda")
    cil.cil_simulate_patterns(w["model"], st2, cil.make_problems(sub_ns, w["L"], [nus[b] for b in sample],
                                                                 [ps[b] for b in sample]), w["dt"], 300,
                              check_every=300)
    outs, _, _, _ = oracle_mod.imex_run(w["model"], [ps[b] for b in sample], [nus[b] for b in sample], sub_ns,
                                        w["L"], w["dt"], 300, 0.0, 300, state=split(sflat, sub_ns), nthreads=8)
    g = split(st2.double().cpu().numpy(), sub_ns)
    for k, b in enumerate(sample):
        assert rel_err(g[k], outs[k]) <= 1e-4, (b, sub_ns[k])
