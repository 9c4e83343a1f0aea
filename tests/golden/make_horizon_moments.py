"""Writes horizon_moments.json: the oracle's feature mean and covariance at
the configured horizons of two FP32 workloads, for the GPU tests that hold the
batched FP32 path to within 2 % of them.  Calls only the oracle (and the
seeded input generators); run from the repository root:

    python tests/golden/make_horizon_moments.py

* fhn128_t100: the first two proposals of the synthetic-likelihood workload
  (FitzHugh-Nagumo 128 x 128, 64 initial states each, T = 100 at dt = 0.05),
  each proposal's statistic as Alg. 3bst forms it: radii fitted to the range
  of distances between distinct synthetic patterns (Sec. 3.2), resample
  vectors C(R, s1, s2) over the index lists of the workload.
* bz_uneven_t100: the first 192 solves of the uneven Brusselator workload
  (sides 32, 64, 128 in turn, per-solve parameters; 2000 steps of dt = 0.05),
  per side the statistic of Alg. 2bst over the two halves of its 64 patterns
  (13 radii from the cross-pair range, 200 resamples).

The initial states are rounded to FP32 first, as the FP32 path receives them.
Beside the moments: per solve the oracle pattern's Euclidean norm; the
moments' deviation when the oracle's own patterns are only stored as FP32
(rounded once, same radii and resamples): how far storage precision alone
moves the statistic; and for the FitzHugh-Nagumo cases the moments'
deviation between the oracle's banded-Cholesky run and a dense cosine-mode
FP64 run of the same IMEX-Euler step (App. B.1.1's operator diagonalised by
the DCT-II basis; written here, as the oracle pins do): the spread of two
correct FP64 solvers at this horizon.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import cil_synth as cs  # noqa: E402
import oracle  # noqa: E402

THREADS = int(os.environ.get("ORACLE_THREADS", "8"))
FHN_PROPOSALS = 2
BZ_SOLVES, BZ_M, BZ_BOOT, BZ_BOOT_SEED = 192, 13, 200, 41


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def rel_moments(Y, mu, Sig):
    m2, S2 = oracle.mean_cov(Y)
    return [float(np.linalg.norm(m2 - mu) / np.linalg.norm(mu)), float(np.linalg.norm(S2 - Sig) / np.linalg.norm(Sig))]


def fhn128_case(p: int):
    w = cs.WORKLOADS["fhn128_mcmc"]
    n, nsyn, nset, nboot, M = w["n"], w["n_syn"], w["n_set"], w["n_boot"], w["M"]
    thetas = cs.relative_draws(w["theta0"], w["window"], w["rel"], seed=w["proposal_seed"])
    par = (thetas[p][0], thetas[p][1], w["alpha"])
    base = oracle.homogeneous_state(w["model"], (w["theta0"][0], w["theta0"][1], w["alpha"]))
    ics = f32(cs.initial_conditions(base, n, nsyn, seed=w["ic_seed"] + p))
    t = time.time()
    out, _, _, stat = oracle.imex_run(w["model"], par, w["nu"], n, w["L"], w["dt"], w["max_steps"], 0.0,
                                      w["max_steps"], state=ics, nthreads=THREADS)
    assert np.all(stat == 0)
    S = out.reshape(nsyn, 2 * n * n)
    lo, hi = oracle.distance_range(S, S, exclude_diagonal=True, nthreads=THREADS)
    radii = oracle.radii_ladder(lo, hi, M)
    D = oracle.pair_d2(S, S, nthreads=THREADS)
    i1, i2, _ = cs.resample_synthetic(nsyn, nset, nboot, seed=w["boot_seed"] + p)
    _, Y = oracle.bootstrap_vectors(D, i1, i2, radii, nthreads=THREADS)
    mu, Sig = oracle.mean_cov(Y)
    S32 = f32(S)
    _, Y32 = oracle.bootstrap_vectors(oracle.pair_d2(S32, S32, nthreads=THREADS), i1, i2, radii, nthreads=THREADS)
    storage = rel_moments(Y32, mu, Sig)
    # the same run by the dense cosine-mode solve, FP64
    h = w["L"] / (n - 1)
    k = np.arange(n)
    V = np.cos(np.pi * k[:, None] * (k + 0.5) / n)
    V /= np.sqrt((V * V).sum(1, keepdims=True))
    lam = (4.0 / h ** 2) * np.sin(np.pi * k / (2 * n)) ** 2
    dt, (mu_, eps_, alpha) = w["dt"], par
    div = [1.0 / (1.0 + dt * w["nu"][s] * (lam[:, None] + lam[None, :])) for s in range(2)]
    cst = ics.copy()
    for _ in range(w["max_steps"]):
        v, u = cst[:, 0], cst[:, 1]
        rv = v + dt * (eps_ * (u - alpha * v))
        ru = u + dt * (-v + mu_ * u - u * u * u)
        cst = np.stack([V.T @ ((V @ rv @ V.T) * div[0]) @ V, V.T @ ((V @ ru @ V.T) * div[1]) @ V], 1)
    C = cst.reshape(nsyn, 2 * n * n)
    _, Yc = oracle.bootstrap_vectors(oracle.pair_d2(C, C, nthreads=THREADS), i1, i2, radii, nthreads=THREADS)
    spread = rel_moments(Yc, mu, Sig)
    print("fhn128 proposal %d: %.0f s, FP64 solver spread (mean, cov) %s, FP32 storage %s"
          % (p, time.time() - t, spread, storage), flush=True)
    return dict(proposal=p, radii=radii.tolist(), mu=mu.tolist(), cov=Sig.tolist(),
                norms=np.linalg.norm(S, axis=1).tolist(), fp64_solver_spread=spread, fp32_storage_spread=storage)


def bz_case():
    w = cs.WORKLOADS["bz_uneven2048"]
    ns, ps, nus = cs.brusselator_uneven(w["count"], w["seed"], sides=w["sides"], rel=w["rel"])
    bases = [oracle.homogeneous_state(w["model"], q) for q in ps]
    flat = f32(cs.uneven_initial_states(bases, ns, seed=w["ic_seed"]))
    off = np.cumsum([0] + [2 * m * m for m in ns])
    cases = []
    for side in w["sides"]:
        sel = [b for b in range(BZ_SOLVES) if ns[b] == side]
        states = [flat[off[b]:off[b + 1]].reshape(2, side, side) for b in sel]
        t = time.time()
        outs, _, _, stat = oracle.imex_run(w["model"], [ps[b] for b in sel], [nus[b] for b in sel], [side] * len(sel),
                                           w["L"], w["dt"], w["max_steps"], 0.0, w["max_steps"], state=states,
                                           nthreads=THREADS)
        assert np.all(np.asarray(stat) == 0)
        P = np.stack([np.asarray(o).reshape(-1) for o in outs])
        half = len(sel) // 2
        D = oracle.pair_d2(P[:half], P[half:], nthreads=THREADS)
        radii = oracle.radii_ladder(D.min(), D.max(), BZ_M)
        ia, ib = cs.resample_halves(half, half, half, half, BZ_BOOT, seed=BZ_BOOT_SEED)
        _, Y = oracle.bootstrap_vectors(D, ia, ib, radii, nthreads=THREADS)
        mu, Sig = oracle.mean_cov(Y)
        P32 = f32(P)
        _, Y32 = oracle.bootstrap_vectors(oracle.pair_d2(P32[:half], P32[half:], nthreads=THREADS), ia, ib, radii,
                                          nthreads=THREADS)
        storage = rel_moments(Y32, mu, Sig)
        print("bz side %d: %d solves, %.0f s, FP32 storage %s" % (side, len(sel), time.time() - t, storage), flush=True)
        cases.append(dict(side=side, solves=sel, radii=radii.tolist(), mu=mu.tolist(), cov=Sig.tolist(),
                          norms=np.linalg.norm(P, axis=1).tolist(), fp32_storage_spread=storage))
    return cases


def main():
    out = dict(
        note="written by tests/golden/make_horizon_moments.py from the oracle only",
        fhn128_t100=[fhn128_case(p) for p in range(FHN_PROPOSALS)],
        bz_uneven_t100=dict(solves=BZ_SOLVES, M=BZ_M, n_boot=BZ_BOOT, boot_seed=BZ_BOOT_SEED, sides=bz_case()),
    )
    with open(os.path.join(HERE, "horizon_moments.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
