"""Seeded synthetic inputs for the CIL hot path.

This module is the only code that both the oracle side (tests) and the product
side (benchmark, smoke check) use.  It draws random numbers and lays them out;
it holds none of the method's arithmetic: steady states, kinetics, distances,
radii and statistics are computed elsewhere, separately on each side.

Generator: numpy's PCG64 seeded with the stated integer.  Draw order for
initial conditions: solve, then species, then row-major grid point.

Workload shapes follow the paper's experiments (Table exp1: 64x64 grids,
M = 13 radii, N_set = 50, N_syn = 1000, n_CIL = 1000) scaled to the benchmark
configurations listed in WORKLOADS.
"""
from __future__ import annotations

import numpy as np

# model ids (same numbering on both sides of the boundary)
FHN, GM, GM_SOURCE, BRUSSELATOR, HEAT = 0, 1, 2, 3, 4


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def initial_conditions(base, n: int, count: int, seed: int, law: str = "additive_pos",
                       delta: float = 1e-2, dtype=np.float64) -> np.ndarray:
    """Initial states [count, 2, n, n]: a base state plus uniform noise.

    ``base``: (v0, w0) or an array [count, 2] of per-solve base values.
    ``law``: "additive_pos"  base + U(0, delta)            (Sec. 4.1)
             "additive_sym"  base + U(-delta, delta)
             "multiplicative" base * (1 + U(-delta, delta)).
    """
    g = rng(seed)
    base = np.asarray(base, dtype=np.float64)
    if base.ndim == 1:
        base = np.broadcast_to(base, (count, 2))
    u = g.random((count, 2, n, n))
    if law == "additive_pos":
        x = base[:, :, None, None] + delta * u
    elif law == "additive_sym":
        x = base[:, :, None, None] + delta * (2.0 * u - 1.0)
    elif law == "multiplicative":
        x = base[:, :, None, None] * (1.0 + delta * (2.0 * u - 1.0))
    else:
        raise ValueError(law)
    return np.ascontiguousarray(x, dtype=dtype)


def cosine_mode(n: int, k: int, l: int) -> np.ndarray:
    """Grid function cos(pi k (i+1/2)/n) cos(pi l (j+1/2)/n) (test input)."""
    i = np.arange(n)
    return np.outer(np.cos(np.pi * k * (i + 0.5) / n), np.cos(np.pi * l * (i + 0.5) / n))


def relative_draws(center, count: int, rel: float, seed: int) -> np.ndarray:
    """Parameter vectors center * (1 + U(-rel, rel)), one row per draw."""
    g = rng(seed)
    c = np.asarray(center, dtype=np.float64)
    return c[None, :] * (1.0 + rel * (2.0 * g.random((count, c.size)) - 1.0))


def resample_halves(nA: int, nB: int, kA: int, kB: int, n_boot: int, seed: int):
    """Alg. 2bst step 2.1 index lists: per resample, kA draws with replacement
    from range(nA) and kB draws with replacement from range(nB)."""
    g = rng(seed)
    ia = g.integers(0, nA, size=(n_boot, kA), dtype=np.int64).astype(np.int32)
    ib = g.integers(0, nB, size=(n_boot, kB), dtype=np.int64).astype(np.int32)
    return ia, ib


def resample_synthetic(n_syn: int, n_set: int, n_boot: int, seed: int):
    """Alg. 3bst index lists.  Per resample: s1 = n_set draws with replacement
    from range(n_syn); s2 = n_syn - n_set draws with replacement from the
    indices not drawn into s1.  Also one subset of n_syn - n_set indices drawn
    without replacement (step 4).  Returns (idx1, idx2, subset)."""
    g = rng(seed)
    k2 = n_syn - n_set
    idx1 = np.empty((n_boot, n_set), dtype=np.int32)
    idx2 = np.empty((n_boot, k2), dtype=np.int32)
    for r in range(n_boot):
        a = g.integers(0, n_syn, size=n_set)
        rest = np.setdiff1d(np.arange(n_syn), a)
        idx1[r] = a
        idx2[r] = rest[g.integers(0, rest.size, size=k2)]
    subset = g.permutation(n_syn)[:k2].astype(np.int32)
    return idx1, idx2, subset


def stripe_patterns(count: int, n: int, seed: int, ring: float = 8.0, modes: int = 12,
                    dtype=np.float32) -> np.ndarray:
    """Stand-in stationary patterns [count, 2, n, n] for feature-only
    workloads: per pattern and species, tanh of a random-signed sum of cosine
    modes whose wave numbers lie on a ring |k| ~ ring (a Turing-like spectrum),
    with the second species a scaled copy plus its own small modes."""
    g = rng(seed)
    i = (np.arange(n) + 0.5) / n
    out = np.empty((count, 2, n, n), dtype=np.float64)
    for c in range(count):
        for s in range(2):
            f = np.zeros((n, n))
            for _ in range(modes):
                ang = g.random() * np.pi / 2
                kx, ky = ring * np.cos(ang), ring * np.sin(ang)
                kx, ky = max(0, int(round(kx))), max(0, int(round(ky)))
                sign = 1.0 if g.random() < 0.5 else -1.0
                f += sign * np.outer(np.cos(np.pi * kx * i), np.cos(np.pi * ky * i))
            out[c, s] = np.tanh(1.5 * f / np.sqrt(modes)) * (1.0 if s == 0 else 0.5)
    return np.ascontiguousarray(out, dtype=dtype)


def turing_unstable_bz(A: float, B: float, Du: float, Dv: float, n: int, L: float = 1.0) -> bool:
    """Input-recipe filter for Brusselator parameter draws: the homogeneous
    state (A, B/A) is stable without diffusion (trace < 0, det > 0 of the
    kinetic Jacobian [[B - 1, A^2], [-B, -A^2]]) and some mode of the grid's
    five-point Laplacian (eigenvalue Lam = lam_k + lam_l, lam_k = 4 sin^2(pi k
    / 2n) / h^2, h = L/(n-1)) grows: det(J - Lam diag(Du, Dv)) < 0."""
    tr, det = B - 1.0 - A * A, A * A
    if not (tr < 0.0 and det > 0.0):
        return False
    h = L / (n - 1)
    lam = 4.0 * np.sin(np.pi * np.arange(n) / (2.0 * n)) ** 2 / (h * h)
    Lam = (lam[:, None] + lam[None, :]).ravel()
    dets = (B - 1.0 - Lam * Du) * (-A * A - Lam * Dv) + A * A * B
    return bool(np.any(dets < 0.0))


def brusselator_uneven(count: int, seed: int, sides=(32, 64, 128), L: float = 1.0, rel: float = 0.05,
                       theta0=(4.5, 6.96, 0.0016, 0.0132)):
    """Per-solve Brusselator problems around a Turing point: solve b has grid
    side sides[b mod len(sides)] and (A, B, Du, Dv) = theta0 (1 + U(-rel, rel))
    drawn until the draw is Turing-unstable on that grid.  Returns the lists
    (sides, params [(A, B)], nus [(Du, Dv)])."""
    g = rng(seed)
    t0 = np.asarray(theta0, dtype=np.float64)
    ns, ps, nus = [], [], []
    while len(ns) < count:
        n = sides[len(ns) % len(sides)]
        A, B, Du, Dv = t0 * (1.0 + g.uniform(-rel, rel, 4))
        if turing_unstable_bz(A, B, Du, Dv, n, L):
            ns.append(n)
            ps.append((A, B))
            nus.append((Du, Dv))
    return ns, ps, nus


def uneven_initial_states(bases, ns, seed: int, delta: float = 1e-2) -> np.ndarray:
    """Concatenated [species][n][n] states of solves of different sides: the
    solve's homogeneous state + U(0, delta) per point (draw order: solve,
    species, row-major), FP64."""
    g = rng(seed)
    out = []
    for base, n in zip(bases, ns):
        noise = g.uniform(0.0, delta, size=(2, n, n))
        out.append((np.asarray(base, dtype=np.float64)[:, None, None] + noise).reshape(-1))
    return np.concatenate(out) if out else np.zeros(0)


# --------------------------------------------------------------------------
# Workload configurations.  Parameter values from Table exp1 where the paper
# gives them; the source form of Gierer-Meinhardt and its Turing parameters are
# the stationarity workload's own definition.

WORKLOADS = {
    # Plain FP64 method: FHN 32x32, fixed 5000 steps, two 64-pattern sets.
    "fhn32_fixed5000": dict(
        model=FHN, params=(1.0, 10.0, 1.0), nu=(0.05, 0.00028), n=32, L=1.0, dt=0.01,
        max_steps=5000, tol=0.0, check_every=5000, count=64, seeds=(1, 2),
        ic_law="additive_sym", radii_base=1.2, M=16),
    # Gierer-Meinhardt with source, 64x64, 500 ICs, run to residual < 1e-8.
    "gm_source64_stationary": dict(
        model=GM_SOURCE, params=(0.5, 1.0), nu=(1.0, 100.0), n=64, L=120.0, dt=0.2,
        max_steps=20000, tol=1e-8, check_every=25, count=500, seeds=(3,),
        ic_law="multiplicative", M=13, n_boot=200),
    # Features alone: 4096 FP32 stand-in patterns of side 128 (d = 32768),
    # halves of 2048, 32 power-law radii, 200 bootstrap resamples of the halves.
    "features4096": dict(count=4096, n=128, M=32, n_boot=200, seeds=(5,), boot_seed=6),
    # Multi-feature CIL (Sec. 3.1): 500 stand-in patterns of side 64, halves of
    # 250, the six norms of Sec. 3.1 with 10 radii each (a 60-entry vector), 200
    # bootstrap resamples; optionally min-max scaled (Sec. 5).
    "mcil_stripes64": dict(count=500, n=64, L=1.0, M=10, n_boot=200, seed=23, boot_seed=24),
    # Uneven batch: 2048 Brusselator solves, sides 32/64/128 in turn, each with
    # its own (A, B, Du, Dv) around Table exp1's point, FP32, T = 100 at dt = 0.05.
    "bz_uneven2048": dict(model=BRUSSELATOR, count=2048, sides=(32, 64, 128), L=1.0, dt=0.05, max_steps=2000,
                          check_every=2000, seed=4, ic_seed=4, rel=0.05),
    # Synthetic-likelihood evaluations for MCMC (Alg. 3bst): FitzHugh-Nagumo
    # 128^2, proposals (mu, eps) = theta0 (1 +- 10 %), 64 synthetic patterns
    # each (T = 100, FP32), 8 data patterns at theta0, 200 resamples, 13
    # adaptive power-law radii; timed on a window of the first 20 proposals.
    "fhn128_mcmc": dict(model=FHN, n=128, L=1.0, nu=(0.05, 0.00028), theta0=(1.0, 10.0), alpha=1.0, rel=0.1,
                        proposals=1000, window=20, n_syn=64, n_set=8, n_boot=200, M=13, dt=0.05, max_steps=2000,
                        proposal_seed=7, data_seed=8, ic_seed=100, boot_seed=9),
}
