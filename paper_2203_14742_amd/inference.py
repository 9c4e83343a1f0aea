"""Parameter inference on top of the batched synthetic likelihood.

`SyntheticCIL` evaluates the cost f(theta) of Alg. 3bst (synthetic CIL,
eq. cil:CF_synth) for a batch of proposals at once: all proposals' synthetic
patterns in one simulate call, then per proposal the adaptive radii (Sec. 3.2)
of its synthetic self-pairs, the resample vectors, the observed vector of the
data set against the synthetic patterns, and one batched likelihood call.
Common random numbers: every proposal uses the same initial-state seeds and
resample index lists, so costs of nearby proposals differ by the model only.

`differential_evolution` is the DE/rand/1/bin optimiser the paper uses to
locate the cost minimum before sampling (Sec. 5: 20 candidates, 50
generations); each generation is one batched evaluation.

`adaptive_metropolis` samples the posterior with adaptive Metropolis
(Haario, Saksman and Tamminen 2001), optionally with a delayed-rejection
second stage (DRAM: Haario, Laine, Mira and Saksman 2006), the samplers the
paper runs on the synthetic likelihood (Sec. 2 and Sec. 5).  K chains advance
together so that each step is one batched evaluation of K proposals (and one
more of the second-stage proposals of the chains whose first stage was
rejected).

Host orchestration only: every step of the statistic runs in the library's
kernels (`paper_2203_14742_amd` calls).
"""
from __future__ import annotations

import numpy as np

from . import (CIL_EINVAL, CIL_SOLVE_NONFINITE, CilError, cil_bootstrap_features, cil_gaussian_loglik, cil_pair_bins,
               cil_pair_bins_adaptive, cil_simulate_patterns, make_problems)


class SyntheticCIL:
    def __init__(self, model: int, n: int, L: float, nu, params_of_theta, data, n_syn: int, n_boot: int, M: int,
                 dt: float, steps: int, ic_states, resample_index_lists, dtype=None):
        """params_of_theta(theta) -> the model's parameter tuple for proposal theta;
        data: device tensor [n_set, 2 n^2] (the observed patterns);
        ic_states: host array [n_syn, 2, n, n] (initial states shared by all proposals);
        resample_index_lists: (s1 [n_boot, n_set], s2 [n_boot, n_syn - n_set], subset
        [n_syn - n_set]) as `cil_synth.resample_synthetic` returns them; the subset
        indexes the synthetic patterns the observed vector pairs with the data set."""
        import torch
        self.model, self.n, self.L, self.nu = model, n, L, nu
        self.params_of_theta = params_of_theta
        self.data = data
        self.n_syn, self.n_boot, self.M, self.dt, self.steps = n_syn, n_boot, M, dt, steps
        self.dtype = dtype or data.dtype
        self.ic = torch.tensor(np.asarray(ic_states), dtype=self.dtype, device=data.device)
        a, b, c = resample_index_lists
        self.idx = (torch.from_numpy(a).to(data.device), torch.from_numpy(b).to(data.device),
                    torch.from_numpy(c)[None, :].to(data.device))
        self.ident = torch.arange(data.shape[0], dtype=torch.int32, device=data.device)[None, :]

    def simulate(self, thetas):
        """The synthetic patterns of every proposal: device tensor
        [P n_syn, 2 n^2], proposal-major, from one simulate call.  Sets
        `last_nonfinite` [P]: proposals with a solve that went non-finite."""
        thetas = np.atleast_2d(np.asarray(thetas, dtype=np.float64))
        P, ns = thetas.shape[0], self.n_syn
        params = [self.params_of_theta(t) for t in thetas for _ in range(ns)]
        st = self.ic.repeat(P, 1, 1, 1).contiguous()
        rep = cil_simulate_patterns(self.model, st, make_problems(self.n, self.L, self.nu, params), self.dt,
                                    self.steps, check_every=max(self.steps, 1), raise_on_nonfinite=False)
        self.last_nonfinite = (rep["status"] == CIL_SOLVE_NONFINITE).reshape(P, ns).any(axis=1)
        return st.reshape(P * ns, 2 * self.n * self.n)

    def costs_from_patterns(self, S):
        """f(theta) per proposal and the log-likelihoods, from the synthetic
        patterns S [P n_syn, 2 n^2] (proposal-major).  np.inf and -np.inf
        where the covariance is not positive definite, and where the
        proposal's distinct synthetic patterns give no radius ladder (Sec. 3.2
        fits the radii between the smallest and largest distance: two equal
        patterns, or all distances equal, leave no range)."""
        import torch
        ns = self.n_syn
        P = S.shape[0] // ns
        Y = torch.empty((P, self.n_boot, self.M), dtype=torch.float64, device=S.device)
        yobs = torch.empty((P, self.M), dtype=torch.float64, device=S.device)
        ok = np.ones(P, dtype=bool)
        for p in range(P):
            Sp = S[p * ns:(p + 1) * ns]
            try:
                _, _, radii, bins, _ = cil_pair_bins_adaptive(Sp, Sp, self.M, exclude_diagonal=True)
            except CilError as e:
                if e.code != CIL_EINVAL:
                    raise
                # the arguments were checked before: the range is degenerate
                ok[p] = False
                continue
            _, Y[p] = cil_bootstrap_features(bins, self.idx[0], self.idx[1], self.M, want_counts=False)
            dbins, _ = cil_pair_bins(self.data, Sp, radii, want_counts=False)
            _, yobs[p] = cil_bootstrap_features(dbins, self.ident, self.idx[2], self.M, want_counts=False)
        f, ll = np.full(P, np.inf), np.full(P, -np.inf)
        good = np.flatnonzero(ok)
        if good.size:
            gi = torch.from_numpy(good).to(S.device)
            fg, lg, _, status = cil_gaussian_loglik(Y[gi].contiguous(), yobs[gi].contiguous())
            fg, lg, status = fg.cpu().numpy(), lg.cpu().numpy(), status.cpu().numpy()
            f[good] = np.where(status == 0, fg, np.inf)
            ll[good] = np.where(status == 0, lg, -np.inf)
        self.last_degenerate = ~ok
        return f, ll

    def costs(self, thetas):
        """f(theta) and the log-likelihoods of a batch of proposals; a
        proposal with a non-finite synthetic pattern gets f = inf and
        loglik = -inf, the others are evaluated as usual."""
        import torch
        S = self.simulate(thetas)
        bad = self.last_nonfinite
        P = bad.size
        f, ll = np.full(P, np.inf), np.full(P, -np.inf)
        good = np.flatnonzero(~bad)
        if good.size == P:
            return self.costs_from_patterns(S)
        if good.size:
            rows = S.reshape(P, self.n_syn, -1)[torch.from_numpy(good).to(S.device)].reshape(good.size * self.n_syn, -1)
            f[good], ll[good] = self.costs_from_patterns(rows.contiguous())
        return f, ll


def differential_evolution(cost_batch, bounds, pop: int = 20, generations: int = 50, F: float = 0.8,
                           CR: float = 0.9, seed: int = 0):
    """DE/rand/1/bin: per target i, mutant x_r1 + F (x_r2 - x_r3) (r1, r2, r3
    distinct and != i, clipped to the bounds), binomial crossover with rate CR
    (one coordinate always from the mutant), greedy selection.  cost_batch(X)
    returns the costs of all rows of X at once.  Returns the best point, its
    cost and the best cost after every generation."""
    lo, hi = (np.asarray(b, dtype=np.float64) for b in zip(*bounds))
    dim = lo.size
    if pop < 4:
        raise ValueError("DE needs pop >= 4")
    g = np.random.default_rng(seed)
    X = lo + (hi - lo) * g.random((pop, dim))
    fX = np.asarray(cost_batch(X), dtype=np.float64)
    history = [float(fX.min())]
    for _ in range(generations):
        T = np.empty_like(X)
        for i in range(pop):
            r1, r2, r3 = g.choice([k for k in range(pop) if k != i], 3, replace=False)
            v = np.clip(X[r1] + F * (X[r2] - X[r3]), lo, hi)
            mask = g.random(dim) < CR
            mask[g.integers(dim)] = True
            T[i] = np.where(mask, v, X[i])
        fT = np.asarray(cost_batch(T), dtype=np.float64)
        better = fT <= fX
        X[better], fX[better] = T[better], fT[better]
        history.append(float(fX.min()))
    b = int(np.argmin(fX))
    return dict(x=X[b].copy(), f=float(fX[b]), history=history, population=X, costs=fX)


def _gauss_log_ratio(y, a, b, Linv):
    """log N(y; a, C) - log N(y; b, C) for one covariance C = L L^T, Linv = L^-1."""
    za, zb = Linv @ (y - a), Linv @ (y - b)
    return -0.5 * (za @ za - zb @ zb)


def adaptive_metropolis(loglik_batch, x0, n_steps: int, C0, bounds=None, seed: int = 0, adapt_start: int = 100,
                        sd: float | None = None, eps: float = 1e-10, dr_scale: float | None = None):
    """K chains of adaptive Metropolis, started at the rows of x0 [K, dim].

    Step t of each chain proposes y = x + L_t z, z ~ N(0, I), C_t = L_t L_t^T:
    C_t = C0 while t <= max(adapt_start, 1), afterwards sd (Cov(x_0 .. x_{t-1}) + eps I)
    with sd = 2.4^2 / dim by default (the chain's own history, updated
    recursively).  Accept with probability min(1, pi(y) / pi(x)) under a flat
    prior inside `bounds` (a proposal outside has pi = 0 and is not
    evaluated).  With dr_scale set, a rejected first stage tries
    y2 = x + dr_scale L_t z2 and accepts it with the delayed-rejection
    probability
        min(1, pi(y2) q(y2 -> y1) (1 - a(y2, y1)) / (pi(x) q(x -> y1) (1 - a(x, y1)))),
    a(u, v) = min(1, pi(v) / pi(u)), q the first-stage Gaussian kernel.

    loglik_batch(X) returns log pi of all rows of X at once (-inf allowed).
    Returns dict(chains [K, n_steps + 1, dim], loglik [K, n_steps + 1],
    accepted [K] first-stage acceptances, accepted_dr [K] second-stage ones,
    evaluations: the number of batched calls made)."""
    x0 = np.atleast_2d(np.asarray(x0, dtype=np.float64))
    K, dim = x0.shape
    C0 = np.atleast_2d(np.asarray(C0, dtype=np.float64))
    if C0.shape != (dim, dim):
        raise ValueError("C0 must be dim x dim")
    sd = 2.4 ** 2 / dim if sd is None else float(sd)
    if bounds is None:
        lo, hi = np.full(dim, -np.inf), np.full(dim, np.inf)
    else:
        lo, hi = (np.asarray(b, dtype=np.float64) for b in zip(*bounds))
    g = np.random.default_rng(seed)
    chains = np.empty((K, n_steps + 1, dim))
    ll = np.empty((K, n_steps + 1))
    chains[:, 0] = x0
    ll[:, 0] = np.asarray(loglik_batch(x0), dtype=np.float64)
    calls = 1
    mean = x0.copy()
    M2 = np.zeros((K, dim, dim))                      # sum of outer products of deviations (Welford)
    acc = np.zeros(K, dtype=np.int64)
    acc_dr = np.zeros(K, dtype=np.int64)
    L0 = np.linalg.cholesky(C0)

    def evaluate(Y, live):
        out = np.full(Y.shape[0], -np.inf)
        if live.any():
            nonlocal calls
            out[live] = np.asarray(loglik_batch(Y[live]), dtype=np.float64)
            calls += 1
        return out

    for t in range(1, n_steps + 1):
        x, lx = chains[:, t - 1], ll[:, t - 1]
        if t <= max(adapt_start, 1):                  # a covariance needs two history points
            Ls = np.broadcast_to(L0, (K, dim, dim))
        else:
            Ls = np.linalg.cholesky(sd * (M2 / (t - 1) + eps * np.eye(dim)))
        y1 = x + np.einsum("kij,kj->ki", Ls, g.standard_normal((K, dim)))
        inside = np.all((y1 >= lo) & (y1 <= hi), axis=1)
        l1 = evaluate(y1, inside)
        with np.errstate(invalid="ignore"):
            log_a1 = np.minimum(0.0, l1 - lx)
        u = np.log(g.random(K))
        take = u < log_a1
        new, lnew = np.where(take[:, None], y1, x), np.where(take, l1, lx)
        acc += take
        if dr_scale is not None:
            rej = ~take
            y2 = x + dr_scale * np.einsum("kij,kj->ki", Ls, g.standard_normal((K, dim)))
            inside2 = rej & np.all((y2 >= lo) & (y2 <= hi), axis=1)
            l2 = evaluate(y2, inside2)
            u2 = np.log(g.random(K))
            for k in np.flatnonzero(inside2):
                if not np.isfinite(l2[k]):
                    continue
                a_y2 = min(1.0, np.exp(min(0.0, l1[k] - l2[k]))) if np.isfinite(l1[k]) else 0.0
                if a_y2 >= 1.0:
                    continue                          # the reverse move would have been taken: ratio 0
                a_x = np.exp(log_a1[k]) if np.isfinite(log_a1[k]) else 0.0
                Linv = np.linalg.inv(Ls[k])
                log_r = (l2[k] - lx[k] + _gauss_log_ratio(y1[k], y2[k], x[k], Linv)
                         + np.log1p(-a_y2) - np.log1p(-a_x))
                if u2[k] < min(0.0, log_r):
                    new[k], lnew[k] = y2[k], l2[k]
                    acc_dr[k] += 1
        chains[:, t], ll[:, t] = new, lnew
        d = new - mean                                # Welford update of the history's mean and scatter
        mean += d / (t + 1)
        M2 += np.einsum("ki,kj->kij", d, new - mean)
    return dict(chains=chains, loglik=ll, accepted=acc, accepted_dr=acc_dr, evaluations=calls)
