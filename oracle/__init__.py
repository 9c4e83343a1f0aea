"""Plain FP64 CPU oracle for the CIL hot path (arXiv 2203.14742).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the HIP path.  Heavy loops (IMEX-Euler and second-order
IMEX stepping with a banded Cholesky diffusion solve, canonical distances,
counts, bootstrap counts) live
in ``cil_oracle.c``; the small statistics (radii ladder, mean/covariance,
Cholesky, cost) are written out here with plain loops.

Every function names the passage of the paper it follows; where the paper is
silent, the docstring states the reading taken.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cil_oracle.c")
_LIB = os.path.join(_HERE, "libcil_oracle.so")

FHN, GM, GM_SOURCE, BRUSSELATOR, HEAT = 0, 1, 2, 3, 4
SOLVE_OK, SOLVE_NONFINITE, SOLVE_MAXSTEPS = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_canonical_d2_f64.restype = ctypes.c_double
        L.oracle_canonical_d2_f32.restype = ctypes.c_double
        L.oracle_exact_sum.restype = ctypes.c_double
        L.oracle_homogeneous_state.argtypes = [ctypes.c_int, dp, dp, dp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# Models (Sec. 4.1) and the grid (App. B.1.1)

def params4(p) -> np.ndarray:
    out = np.zeros(4)
    p = list(p)
    out[: len(p)] = p
    return out


def kinetics(model: int, p, v: float, w: float):
    """Reaction terms (f, g) at one point, Sec. 4.1."""
    f = ctypes.c_double()
    g = ctypes.c_double()
    pp = params4(p)
    lib().oracle_kinetics(ctypes.c_int(model), _ptr(pp), ctypes.c_double(v), ctypes.c_double(w),
                          ctypes.byref(f), ctypes.byref(g))
    return f.value, g.value


def homogeneous_state(model: int, p):
    """Spatially homogeneous steady state (v0, w0), Sec. 4.1."""
    pp = params4(p)
    v0 = ctypes.c_double()
    w0 = ctypes.c_double()
    rc = lib().oracle_homogeneous_state(model, pp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        ctypes.byref(v0), ctypes.byref(w0))
    if rc:
        raise ValueError("unknown model")
    return v0.value, w0.value


def mol_rhs(model: int, p, nu, n: int, L: float, state: np.ndarray) -> np.ndarray:
    """Right-hand side of the method-of-lines system, App. B.1.1 (direct stencil)."""
    st = _f64(state).reshape(-1)
    out = np.empty_like(st)
    lib().oracle_mol_rhs(ctypes.c_int(model), _ptr(params4(p)), _ptr(_f64(nu)), ctypes.c_int(n),
                         ctypes.c_double(L), _ptr(st), _ptr(out))
    return out.reshape(2, n, n)


def implicit_diffusion(n: int, L: float, dt: float, nu: float, b: np.ndarray) -> np.ndarray:
    """Solve (I - dt*nu*Lap_h) x = b by banded Cholesky of the stencil matrix."""
    x = _f64(b).reshape(-1).copy()
    rc = lib().oracle_implicit_diffusion(ctypes.c_int(n), ctypes.c_double(L), ctypes.c_double(dt),
                                         ctypes.c_double(nu), _ptr(x))
    if rc:
        raise RuntimeError("implicit diffusion solve failed (%d)" % rc)
    return x.reshape(n, n)


def imex_run(model: int, params, nu, n, L, dt: float, max_steps: int, tol: float = 0.0,
             check_every: int = 1, state: np.ndarray | None = None, nthreads: int = 0, scheme: str = "euler"):
    """IMEX-Euler runs of a batch of solves, one grid side per solve allowed
    (scheme "sbdf2": the second-order IMEX stepper, semi-implicit BDF2 with
    an IMEX-Euler first step).

    ``params``: [B, <=4]; ``nu``: [B, 2]; ``n``, ``L``: scalars or [B];
    ``state``: list of [2, n_b, n_b] arrays or an array [B, 2, n, n] (FP64).
    Returns (states, steps_taken, final_resid, status); states have the input
    layout.
    """
    if isinstance(state, np.ndarray) and state.ndim == 4:
        states = [state[b] for b in range(state.shape[0])]
        stacked = True
    else:
        states = list(state)
        stacked = False
    B = len(states)
    nn = np.broadcast_to(np.asarray(n, dtype=np.int32), (B,)).copy()
    LL = np.broadcast_to(np.asarray(L, dtype=np.float64), (B,)).copy()
    nus = _f64(np.broadcast_to(np.asarray(nu, dtype=np.float64), (B, 2))).copy()
    pp = np.stack([params4(q) for q in np.broadcast_to(np.asarray(params, dtype=np.float64),
                                                       (B, np.asarray(params).shape[-1]))])
    sizes = [2 * int(k) * int(k) for k in nn]
    off = np.zeros(B, dtype=np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    buf = np.concatenate([_f64(s).reshape(-1) for s in states]) if B else np.zeros(0)
    steps = np.zeros(B, dtype=np.int64)
    resid = np.zeros(B, dtype=np.float64)
    status = np.zeros(B, dtype=np.int32)
    if scheme not in ("euler", "sbdf2"):
        raise ValueError(scheme)
    run = lib().oracle_imex_batch if scheme == "euler" else lib().oracle_sbdf2_batch
    rc = run(ctypes.c_int(model), ctypes.c_int(B), _ptr(nn), _ptr(LL), _ptr(nus), _ptr(pp), ctypes.c_double(dt),
             ctypes.c_long(max_steps), ctypes.c_double(tol), ctypes.c_int(check_every), _ptr(buf), _ptr(off),
             _ptr(steps), _ptr(resid), _ptr(status), ctypes.c_int(nthreads))
    if rc:
        raise RuntimeError("oracle IMEX run failed")
    outs = [buf[off[b]: off[b] + sizes[b]].reshape(2, nn[b], nn[b]) for b in range(B)]
    if stacked:
        outs = np.stack(outs)
    return outs, steps, resid, status


def dct_modes_diffusion(n: int, L: float, dt: float, nu: float, b: np.ndarray) -> np.ndarray:
    """Second, independent mode of the implicit diffusion solve, used only to
    cross-check the banded Cholesky: the ghost-copy Neumann Laplacian has the
    cosine eigenvectors cos(pi k (i+1/2)/n) with eigenvalues
    -(4/h^2) sin^2(pi k / 2n); solve by dense O(n^3) separable products."""
    h = L / (n - 1)
    i = np.arange(n)
    k = np.arange(n)[:, None]
    V = np.cos(np.pi * k * (i + 0.5) / n)             # rows = modes
    V /= np.sqrt((V * V).sum(1, keepdims=True))       # orthonormal
    lam = (4.0 / h ** 2) * np.sin(np.pi * np.arange(n) / (2 * n)) ** 2
    Bh = V @ _f64(b) @ V.T
    Bh /= 1.0 + dt * nu * (lam[:, None] + lam[None, :])
    return V.T @ Bh @ V


# --------------------------------------------------------------------------
# Correlation sums (Sec. 2.1 eqs. eCDF, CIL) on the canonical squared distance

def canonical_d2(a: np.ndarray, b: np.ndarray) -> float:
    """D = RN64(sum_k fl64(a_k - b_k)^2), exact sum rounded once."""
    if a.dtype == np.float32:
        a = np.ascontiguousarray(a, np.float32)
        b = np.ascontiguousarray(b, np.float32)
        return lib().oracle_canonical_d2_f32(_ptr(a), _ptr(b), ctypes.c_long(a.size))
    a = _f64(a)
    b = _f64(b)
    return lib().oracle_canonical_d2_f64(_ptr(a), _ptr(b), ctypes.c_long(a.size))


def exact_sum(x: np.ndarray) -> float:
    x = _f64(x)
    return lib().oracle_exact_sum(_ptr(x), ctypes.c_long(x.size))


def _as_set(S):
    S = np.ascontiguousarray(S)
    if S.dtype not in (np.float32, np.float64):
        S = S.astype(np.float64)
    return S.reshape(S.shape[0], -1)


def pair_d2(A, B, nthreads: int = 0) -> np.ndarray:
    """All canonical squared distances D[i, j] between rows of A and rows of B."""
    A = _as_set(A)
    B = _as_set(B)
    if A.dtype != B.dtype:
        raise TypeError("sets must share a dtype")
    D = np.empty((A.shape[0], B.shape[0]))
    lib().oracle_pair_d2(_ptr(A), ctypes.c_long(A.shape[0]), _ptr(B), ctypes.c_long(B.shape[0]),
                         ctypes.c_long(A.shape[1]), ctypes.c_int(int(A.dtype == np.float32)), _ptr(D),
                         ctypes.c_int(nthreads))
    return D


def pair_d2_sampled(A, B, ia, jb, nthreads: int = 0) -> np.ndarray:
    A = _as_set(A)
    B = _as_set(B)
    ia = np.ascontiguousarray(ia, dtype=np.int64)
    jb = np.ascontiguousarray(jb, dtype=np.int64)
    D = np.empty(ia.size)
    lib().oracle_pair_d2_sampled(_ptr(A), _ptr(B), ctypes.c_long(A.shape[1]),
                                 ctypes.c_int(int(A.dtype == np.float32)), _ptr(ia), _ptr(jb),
                                 ctypes.c_long(ia.size), _ptr(D), ctypes.c_int(nthreads))
    return D


def counts_from_d2(D: np.ndarray, radii) -> np.ndarray:
    """c_m = #{pairs : D < fl(R_m * R_m)}, m = 1..M (eq. eCDF numerator)."""
    D = _f64(D).reshape(-1)
    r = _f64(radii)
    c = np.zeros(r.size, dtype=np.int64)
    lib().oracle_counts(_ptr(D), ctypes.c_long(D.size), _ptr(r), ctypes.c_int(r.size), _ptr(c))
    return c


def bins_from_d2(D: np.ndarray, radii) -> np.ndarray:
    """Per pair: the number of radii it lies under, #{m : D < R_m^2}."""
    Df = _f64(D)
    r = _f64(radii)
    out = np.zeros(Df.size, dtype=np.uint8)
    lib().oracle_bins(_ptr(Df), ctypes.c_long(Df.size), _ptr(r), ctypes.c_int(r.size), _ptr(out))
    return out.reshape(np.shape(D))


def cil_vector(A, B, radii, nthreads: int = 0):
    """y_m = C(R_m, A, B) (eqs. eCDF and CIL); returns (counts, y)."""
    D = pair_d2(A, B, nthreads)
    c = counts_from_d2(D, radii)
    return c, c / float(D.size)


def distance_range(A, B, exclude_diagonal: bool = False, nthreads: int = 0):
    """Smallest and largest canonical squared distance over the pairs."""
    D = pair_d2(A, B, nthreads)
    if exclude_diagonal:
        D = D[~np.eye(D.shape[0], D.shape[1], dtype=bool)]
    return float(D.min()), float(D.max())


def radii_ladder(d2min: float, d2max: float, M: int, law: str = "power"):
    """Radii R_1 > ... > R_M from the distance range (Sec. 2.1, Sec. 3.2):
    R_0 = largest distance, R_M = smallest; power law R_m = R_0 b^-m with
    b = (R_0/R_M)^(1/M), or linear R_m = R_0 - m h with h = (R_0 - R_M)/M."""
    R0 = math.sqrt(d2max)
    RM = math.sqrt(d2min)
    if not (R0 > 0.0) or not (RM > 0.0) or not (R0 > RM) or M < 1:
        raise ValueError("degenerate distance range")
    if law == "power":
        b = (R0 / RM) ** (1.0 / M)
        return np.array([R0 * b ** (-m) for m in range(1, M + 1)])
    if law == "linear":
        h = (R0 - RM) / M
        return np.array([R0 - m * h for m in range(1, M + 1)])
    raise ValueError(law)


def power_radii(R0: float, base: float, M: int):
    """R_m = R_0 * base^-m, m = 1..M (Sec. 2.1 power law with a fixed b)."""
    return np.array([R0 * base ** (-m) for m in range(1, M + 1)])


def bootstrap_vectors(D: np.ndarray, idxA, idxB, radii, nthreads: int = 0):
    """Alg. 2bst / 3bst step 2: one correlation integral vector per resample,
    from the pair distances and the resample index lists (repeats allowed).
    Returns (integer counts [n_boot, M], Y [n_boot, M])."""
    D = _f64(D)
    idxA = np.ascontiguousarray(idxA, dtype=np.int32)
    idxB = np.ascontiguousarray(idxB, dtype=np.int32)
    r = _f64(radii)
    nb, kA = idxA.shape
    kB = idxB.shape[1]
    Yc = np.zeros((nb, r.size), dtype=np.int64)
    Y = np.zeros((nb, r.size))
    lib().oracle_bootstrap(_ptr(D), ctypes.c_long(D.shape[1]), _ptr(idxA), ctypes.c_int(kA), _ptr(idxB),
                           ctypes.c_int(kB), ctypes.c_int(nb), _ptr(r), ctypes.c_int(r.size), _ptr(Yc),
                           _ptr(Y), ctypes.c_int(nthreads))
    return Yc, Y


# --------------------------------------------------------------------------
# Gaussian synthetic likelihood (eqs. cil:CF, cil:CF_synth)

def mean_cov(Y: np.ndarray):
    """Two-pass sample mean and covariance with the 1/(n-1) normaliser."""
    Y = _f64(Y)
    n, M = Y.shape
    mu = np.zeros(M)
    for k in range(n):
        mu += Y[k]
    mu /= n
    S = np.zeros((M, M))
    for k in range(n):
        z = Y[k] - mu
        S += np.outer(z, z)
    S /= (n - 1)
    return mu, S


def cholesky(S: np.ndarray) -> np.ndarray:
    """Cholesky-Banachiewicz, row by row.  Raises when a pivot is not above
    M * 2^-52 * S_ii: the matrix is then singular to working precision (an
    exactly rank-deficient covariance leaves pivots of rounding size)."""
    M = S.shape[0]
    L = np.zeros_like(S)
    for i in range(M):
        for j in range(i + 1):
            s = S[i, j]
            for k in range(j):
                s -= L[i, k] * L[j, k]
            if i == j:
                if not (s > M * 2.0 ** -52 * S[i, i]):
                    raise np.linalg.LinAlgError("not positive definite")
                L[i, i] = math.sqrt(s)
            else:
                L[i, j] = s / L[j, j]
    return L


def gaussian_cost(Y: np.ndarray, y_obs: np.ndarray):
    """Cost f = (y - mu)^T Sigma^-1 (y - mu) (eq. cil:CF_synth) and the full
    Gaussian log-likelihood -f/2 - sum log L_ii - (M'/2) log 2 pi, over the
    bins whose sample variance is non-zero (M' of them).

    Returns dict(f, loglik, m_eff, keep, mu, cov, ok)."""
    mu, S = mean_cov(Y)
    keep = np.array([S[m, m] != 0.0 for m in range(S.shape[0])])
    idx = np.flatnonzero(keep)
    Sk = S[np.ix_(idx, idx)]
    d = _f64(y_obs)[idx] - mu[idx]
    out = dict(mu=mu, cov=S, keep=keep, m_eff=int(idx.size))
    try:
        L = cholesky(Sk)
    except np.linalg.LinAlgError:
        out.update(f=float("nan"), loglik=float("nan"), ok=False)
        return out
    z = np.zeros(idx.size)
    for i in range(idx.size):                 # forward substitution L z = d
        s = d[i]
        for k in range(i):
            s -= L[i, k] * z[k]
        z[i] = s / L[i, i]
    f = float(sum(zi * zi for zi in z))
    logdet_half = float(sum(math.log(L[i, i]) for i in range(idx.size)))
    loglik = -0.5 * f - logdet_half - 0.5 * idx.size * math.log(2.0 * math.pi)
    out.update(f=f, loglik=loglik, ok=True)
    return out


# --------------------------------------------------------------------------
# Further pattern features: the multi-feature CIL of Sec. 3.1 (norms
# eqs. norm:L2 ... norm:W1infprime) and the min-max scaling of Sec. 5.

def minmax_scale(patterns: np.ndarray) -> np.ndarray:
    """Sec. 5 min-max normalisation, per pattern and per species:
    (s - min) / (max - min) over the species' grid, evaluated in FP64 and
    rounded once to the input's type.  Reading: a constant species (max ==
    min, the paper divides by zero) becomes 0."""
    X = np.asarray(patterns)          # [count][2][n][n] or [count][2 n^2]
    out = np.empty_like(X)
    flat = X.reshape(X.shape[0], 2, -1)
    res = out.reshape(flat.shape)
    for p in range(flat.shape[0]):
        for c in range(2):
            v = flat[p, c].astype(np.float64)
            lo, hi = v.min(), v.max()
            span = hi - lo
            res[p, c] = ((v - lo) / span).astype(X.dtype) if span > 0.0 else np.zeros(v.shape, dtype=X.dtype)
    return out


def augment(patterns: np.ndarray, n: int, L: float) -> np.ndarray:
    """Sec. 3.1: the Sobolev norms use finite-difference derivatives.  Reading:
    forward differences on the grid of the discretisation (h = L / (n - 1)),
    per species, along x (within a row) and y (across rows), appended to the
    pattern: [s | D_x s | D_y s], each value formed in FP64 and rounded once to
    the input's type.  Then the W^{1,2} distance of two patterns (eq.
    norm:W12) is the L2 distance of their augmented vectors."""
    X = np.asarray(patterns)
    S = X.reshape(-1, 2, n, n)
    h = L / (n - 1)
    s64 = S.astype(np.float64)
    dx = (s64[:, :, :, 1:] - s64[:, :, :, :-1]) / h
    dy = (s64[:, :, 1:, :] - s64[:, :, :-1, :]) / h
    parts = [S.reshape(S.shape[0], -1), dx.astype(X.dtype).reshape(S.shape[0], -1),
             dy.astype(X.dtype).reshape(S.shape[0], -1)]
    return np.concatenate(parts, axis=1)


def pair_maxabs(A, B, seg_end) -> np.ndarray:
    """Eqs. norm:Linf, norm:W1inf, norm:W1infprime: the L-infinity norm of a
    difference, per segment [seg_end[s-1], seg_end[s]) of the vectors:
    D[i, j, s] = max_k |a_k - b_k| with the difference formed in FP64 (0 for an
    empty segment)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    ends = [int(e) for e in seg_end]
    out = np.zeros((A.shape[0], B.shape[0], len(ends)))
    for i in range(A.shape[0]):
        prev = 0
        for s, e in enumerate(ends):
            if e > prev:
                out[i, :, s] = np.abs(B[:, prev:e] - A[i, prev:e]).max(axis=1)
            prev = e
    return out


def combine_segments(D: np.ndarray, mode: int) -> np.ndarray:
    """W^{1,inf} (eq. norm:W1inf: the largest of the per-derivative maxima,
    mode 0), its variant with a sum (eq. norm:W1infprime, mode 1, summed left
    to right in FP64), and the sum-of-L2 W^{1,2} variant (eq. norm:W12prime,
    mode 2: from per-part squared distances, the sum of their square roots,
    left to right)."""
    D = np.asarray(D, dtype=np.float64)
    f = np.sqrt if mode == 2 else (lambda x: x)
    v = f(D[..., 0]).copy()
    for s in range(1, D.shape[-1]):
        v = np.maximum(v, D[..., s]) if mode == 0 else v + f(D[..., s])
    return v


def bins_from_values(V: np.ndarray, radii) -> np.ndarray:
    """Eq. eCDF for distances that are not squared: per pair the number of
    radii it lies under, #{m : V < R_m}."""
    V = np.asarray(V, dtype=np.float64)
    r = np.asarray(radii, dtype=np.float64)
    out = np.zeros(V.shape, dtype=np.uint8)
    for m in range(r.size):
        out += (V < r[m]).astype(np.uint8)
    return out


def counts_from_values(V: np.ndarray, radii) -> np.ndarray:
    """C(R_m) numerators of eq. eCDF for distances: #{pairs : V < R_m}."""
    V = np.asarray(V, dtype=np.float64)
    return np.array([int((V < float(r)).sum()) for r in np.asarray(radii, dtype=np.float64)], dtype=np.int64)
