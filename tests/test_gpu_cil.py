"""GPU parity of the CIL statistic against the FP64 oracle (through the C ABI).

Counts, bins and bootstrap counts are integers: bit-exact.  Canonical
distances are exactly rounded: bit-exact.  Likelihood values: 1e-10 relative.
"""
import math

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


def sets(nA, nB, d, seed, dtype, scale=1.0, offset=0.0):
    g = np.random.default_rng(seed)
    A = (offset + scale * g.standard_normal((nA, d))).astype(dtype)
    B = (offset + scale * g.standard_normal((nB, d))).astype(dtype)
    return A, B


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("d", [1, 37, 2048, 8192])
def test_canonical_distance_bit_exact(cil, oracle_mod, dtype, d):
    A, B = sets(9, 11, d, seed=d, dtype=dtype, offset=0.7)
    ia = np.repeat(np.arange(9), 11)
    jb = np.tile(np.arange(11), 9)
    got = cil.cil_canonical_d2(dev(A), dev(B), torch.from_numpy(ia), torch.from_numpy(jb)).cpu().numpy()
    want = oracle_mod.pair_d2(A, B).reshape(-1)
    assert np.array_equal(got, want)


def test_fp32_ties_need_no_exact_fallback(cil, oracle_mod):
    """FP32 sets have exact squares, so the exact sum has few bits and often
    sits exactly half-way between two doubles.  The double-double sum is then
    exact and certified as such: bit-exact results, no slow exact fallback."""
    g = np.random.default_rng(21)
    A = (20.0 * g.random((40, 8192))).astype(np.float32)
    B = (20.0 * g.random((50, 8192))).astype(np.float32)
    ia = np.repeat(np.arange(40), 50)
    jb = np.tile(np.arange(50), 40)
    got = cil.cil_canonical_d2(dev(A), dev(B), torch.from_numpy(ia), torch.from_numpy(jb)).cpu().numpy()
    assert np.array_equal(got, oracle_mod.pair_d2(A, B).reshape(-1))
    assert cil.cil_last_distance_stats()["exact_fallbacks"] == 0


def test_exact_summation_path_bit_exact(cil, oracle_mod):
    """The rarely needed exact (expansion) summation, forced on every pair."""
    A, B = sets(5, 6, 3001, seed=1, dtype=np.float64, scale=1e3, offset=-2.0)
    ia = np.repeat(np.arange(5), 6)
    jb = np.tile(np.arange(6), 5)
    cil.cil_set_option(cil.CIL_OPT_FORCE_EXACT_SUM, 1)
    try:
        got = cil.cil_canonical_d2(dev(A), dev(B), torch.from_numpy(ia), torch.from_numpy(jb)).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        cil.cil_set_option(cil.CIL_OPT_FORCE_EXACT_SUM, 0)
    assert np.array_equal(got, oracle_mod.pair_d2(A, B).reshape(-1))


def adversarial_sets(case, nA, nB, d, seed):
    g = np.random.default_rng(seed)
    if case == "random":
        A = g.standard_normal((nA, d))
        B = g.standard_normal((nB, d))
    elif case == "offset":                       # large common offset, small spread
        A = 40.0 + 0.01 * g.standard_normal((nA, d))
        B = 40.0 + 0.01 * g.standard_normal((nB, d))
    elif case == "near_equal":                   # B rows are tiny perturbations of A rows
        A = g.standard_normal((nA, d))
        B = A[g.integers(0, nA, nB)] + 1e-5 * g.standard_normal((nB, d))
    elif case == "dynamic_range":                # entries spanning many binades
        A = g.standard_normal((nA, d)) * 10.0 ** g.integers(-6, 4, size=(nA, d))
        B = g.standard_normal((nB, d)) * 10.0 ** g.integers(-6, 4, size=(nB, d))
    elif case == "bf16_boundary":                # values halfway between bf16 neighbours
        base = 2.0 ** g.integers(-3, 3, size=(nA + nB, d))
        mant = (g.integers(128, 256, size=(nA + nB, d)) + 0.5) / 128.0
        X = base * mant * np.where(g.random((nA + nB, d)) < 0.5, -1, 1)
        A, B = X[:nA], X[nA:]
    elif case == "stripes":                      # Turing-like stand-in patterns
        X = cs.stripe_patterns(nA + nB, int(np.sqrt(d // 2)), seed=seed).reshape(nA + nB, -1)
        A, B = X[:nA], X[nA:]
    return A.astype(np.float32), B.astype(np.float32)


@pytest.mark.parametrize("case", ["random", "offset", "near_equal", "dynamic_range", "bf16_boundary", "stripes"])
@pytest.mark.parametrize("d", [200, 2048, 8192])
def test_fast_pass_bound_holds(cil, oracle_mod, case, d):
    """P10: the split-bf16x3 Gram value is within its stated bound of the
    canonical distance for every pair, on random and adversarial inputs; the
    counts after the re-check equal the canonical counts."""
    nA, nB = 40, 37
    if case == "stripes":
        d = {200: 2 * 10 * 10, 2048: 2048, 8192: 8192}[d]
    A, B = adversarial_sets(case, nA, nB, d, seed=d)
    d2, eps = cil.cil_approx_d2(dev(A), dev(B))
    D = oracle_mod.pair_d2(A, B)
    d2, eps = d2.cpu().numpy(), eps.cpu().numpy()
    assert np.all(np.abs(d2 - D) <= eps), float((np.abs(d2 - D) / np.maximum(eps, 1e-300)).max())
    rel = float(np.median(eps / np.maximum(D, 1e-300)))
    print("%s d=%d: median bound/D %.2e, max err/bound %.3f" % (case, d, rel,
          float((np.abs(d2 - D) / np.maximum(eps, 1e-300)).max())))
    radii = oracle_mod.radii_ladder(D.min() if D.min() > 0 else D.max() / 100, D.max(), 13)
    c, _ = cil.cil_features(dev(A), dev(B), radii)
    assert np.array_equal(c, oracle_mod.counts_from_d2(D, radii))


def test_fast_pass_bound_fp64(cil, oracle_mod):
    A, B = adversarial_sets("dynamic_range", 30, 33, 777, seed=1)
    A, B = A.astype(np.float64), B.astype(np.float64)
    d2, eps = cil.cil_approx_d2(dev(A), dev(B))
    D = oracle_mod.pair_d2(A, B)
    assert np.all(np.abs(d2.cpu().numpy() - D) <= eps.cpu().numpy())


@pytest.mark.parametrize("kc", [32, 64, 128])
@pytest.mark.parametrize("case", ["random", "offset", "near_equal", "stripes"])
def test_gram_flush_interval_bound_and_counts(cil, oracle_mod, kc, case):
    """Shorter FP32 accumulation intervals than 256 narrow the stated bound;
    it still holds for every pair and the counts stay exact."""
    nA, nB, d = 40, 37, 8192
    A, B = adversarial_sets(case, nA, nB, d, seed=d + kc)
    D = oracle_mod.pair_d2(A, B)
    try:
        cil.cil_set_option(cil.CIL_OPT_GRAM_FLUSH, 256)
        d2w, epsw = cil.cil_approx_d2(dev(A), dev(B))
        cil.cil_set_option(cil.CIL_OPT_GRAM_FLUSH, kc)
        d2, eps = cil.cil_approx_d2(dev(A), dev(B))
        radii = oracle_mod.radii_ladder(D.min() if D.min() > 0 else D.max() / 100, D.max(), 13)
        c, _ = cil.cil_features(dev(A), dev(B), radii)
        lo, hi, r2, bins, c2 = cil.cil_pair_bins_adaptive(dev(A), dev(B), 13)
    finally:
        cil.cil_set_option(cil.CIL_OPT_GRAM_FLUSH, 64)
    d2, eps = d2.cpu().numpy(), eps.cpu().numpy()
    assert np.all(np.abs(d2 - D) <= eps)
    assert np.all(eps < epsw.cpu().numpy())
    assert np.array_equal(c, oracle_mod.counts_from_d2(D, radii))
    assert (lo, hi) == (D.min(), D.max())
    assert np.array_equal(bins.cpu().numpy(), oracle_mod.bins_from_d2(D, r2))


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("kc", [64, 256])
@pytest.mark.parametrize("nA,nB,d", [(40, 37, 8192), (130, 257, 2048), (1, 300, 64), (300, 1, 200),
                                     (129, 128, 33000), (1000, 1100, 96)])
def test_gram_pipeline_gives_identical_sums(cil, oracle_mod, variant, kc, nA, nB, d):
    """The LDS-DMA pipelined Gram (launch or XCD tile order) computes the same
    products in the same order as the register-staged one: identical
    approximate distances and bounds, on ragged tiles, one-row sets and a
    dimension that is not a multiple of the staging depth."""
    A, B = sets(nA, nB, d, seed=nA + nB + d, dtype=np.float32)
    try:
        cil.cil_set_option(cil.CIL_OPT_GRAM_FLUSH, kc)
        cil.cil_set_option(cil.CIL_OPT_GRAM_PIPELINE, 0)
        d2a, epsa = cil.cil_approx_d2(dev(A), dev(B))
        cil.cil_set_option(cil.CIL_OPT_GRAM_PIPELINE, variant)
        d2b, epsb = cil.cil_approx_d2(dev(A), dev(B))
    finally:
        cil.cil_set_option(cil.CIL_OPT_GRAM_PIPELINE, 2)
        cil.cil_set_option(cil.CIL_OPT_GRAM_FLUSH, 64)
    assert torch.equal(d2a, d2b) and torch.equal(epsa, epsb)
    D = oracle_mod.pair_d2(A, B)
    assert np.all(np.abs(d2b.cpu().numpy() - D) <= epsb.cpu().numpy())


def test_gram_options_reject_other_values(cil):
    for opt, v in ((cil.CIL_OPT_GRAM_FLUSH, 96), (cil.CIL_OPT_GRAM_PIPELINE, 3), (cil.CIL_OPT_GRAM_PIPELINE, -1)):
        with pytest.raises(cil.CilError) as e:
            cil.cil_set_option(opt, v)
        assert e.value.code == cil.CIL_EINVAL


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nA,nB,d,M", [(1, 1, 8, 3), (67, 131, 50, 13), (64, 64, 2048, 16), (130, 70, 333, 32),
                                       (20, 30, 100, 100)])
def test_counts_and_bins_bit_exact(cil, oracle_mod, dtype, nA, nB, d, M):
    A, B = sets(nA, nB, d, seed=nA * 7 + d, dtype=dtype)
    D = oracle_mod.pair_d2(A, B)
    lo, hi = D.min(), D.max()
    if lo == hi:
        lo = hi / 4
    radii = oracle_mod.radii_ladder(lo, hi, M)
    want_c = oracle_mod.counts_from_d2(D, radii)
    want_b = oracle_mod.bins_from_d2(D, radii)
    c, y = cil.cil_features(dev(A), dev(B), radii)
    assert np.array_equal(c, want_c)
    assert np.array_equal(y, want_c / float(nA * nB))
    bins, c2 = cil.cil_pair_bins(dev(A), dev(B), radii)
    assert np.array_equal(bins.cpu().numpy(), want_b)
    assert np.array_equal(c2, want_c)


def test_counts_with_exact_ties(cil, oracle_mod):
    """Integer patterns and integer radii put pairs exactly on radii: the
    re-check decides them with the strict '<'."""
    g = np.random.default_rng(6)
    A = g.integers(-3, 4, size=(40, 7)).astype(np.float64)
    B = g.integers(-3, 4, size=(33, 7)).astype(np.float64)
    radii = np.arange(12, 0, -1).astype(np.float64)
    want = oracle_mod.counts_from_d2(oracle_mod.pair_d2(A, B), radii)
    c, _ = cil.cil_features(dev(A), dev(B), radii)
    assert np.array_equal(c, want)
    st = cil.cil_last_distance_stats()
    assert st["rechecked"] > 0
    c32, _ = cil.cil_features(dev(A.astype(np.float32)), dev(B.astype(np.float32)), radii)
    assert np.array_equal(c32, want)


def test_empty_sets(cil):
    A = torch.zeros((0, 8), dtype=torch.float64, device="cuda")
    B = torch.zeros((5, 8), dtype=torch.float64, device="cuda")
    c, y = cil.cil_features(A, B, [2.0, 1.0])
    assert list(c) == [0, 0]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("excl", [False, True])
def test_distance_range_bit_exact(cil, oracle_mod, dtype, excl):
    A, B = sets(70, 70, 515, seed=3, dtype=dtype)
    if excl:
        B = A.copy()
    got = cil.cil_distance_range(dev(A), dev(B), exclude_diagonal=excl)
    want = oracle_mod.distance_range(A, B, exclude_diagonal=excl)
    assert got == want


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("law", ["power", "linear"])
def test_adaptive_bins_bit_exact(cil, oracle_mod, dtype, law):
    """Range, radii and bins from one fast pass equal the oracle's canonical
    range, its radii ladder and its bins (both radius laws of Sec. 2.1)."""
    A, B = sets(70, 90, 515, seed=8, dtype=dtype)
    M = 16
    lo, hi, radii, bins, counts = cil.cil_pair_bins_adaptive(dev(A), dev(B), M, law=0 if law == "power" else 1)
    D = oracle_mod.pair_d2(A, B)
    assert (lo, hi) == (D.min(), D.max())
    want_r = oracle_mod.radii_ladder(D.min(), D.max(), M, law=law)
    assert np.array_equal(radii, want_r)
    assert np.array_equal(bins.cpu().numpy(), oracle_mod.bins_from_d2(D, want_r))
    assert np.array_equal(counts, oracle_mod.counts_from_d2(D, want_r))


def duplicated_sets(dtype, d=515):
    """Integer sets whose 59 x 59 cross pairs of copies (a against b) all lie
    at the largest distance; row 0 of each set lies near the origin, so its
    pairs are shorter.  More than 2048 pairs then sit at the top of the range,
    or on a radius placed there."""
    g = np.random.default_rng(21)
    a = g.integers(4, 8, size=d)
    b = -g.integers(4, 8, size=d)
    A = np.tile(a, (60, 1)).astype(dtype)
    B = np.tile(b, (60, 1)).astype(dtype)
    A[0] = g.integers(-2, 2, size=d)
    B[0] = g.integers(-2, 2, size=d)
    return A, B


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_range_and_bins_with_long_recheck_lists(cil, oracle_mod, dtype):
    """Re-check lists longer than the first canonical launch covers (3481
    range candidates, 3481 pairs on a radius) finish in the second launch:
    range, radii, bins and counts stay those of the oracle (eqs. eCDF, CIL,
    Sec. 2.1)."""
    A, B = duplicated_sets(dtype)
    D = oracle_mod.pair_d2(A, B)
    assert (D == D.max()).sum() == 59 * 59
    got = cil.cil_distance_range(dev(A), dev(B))
    assert got == (D.min(), D.max())
    assert cil.cil_last_distance_stats()["rechecked"] >= 59 * 59
    radii = np.array([math.sqrt(D.max()), math.sqrt(D.max()) * 0.5, math.sqrt(D.min()) * 0.999])
    bins, counts = cil.cil_pair_bins(dev(A), dev(B), radii)
    assert np.array_equal(bins.cpu().numpy(), oracle_mod.bins_from_d2(D, radii))
    assert np.array_equal(counts, oracle_mod.counts_from_d2(D, radii))
    assert cil.cil_last_distance_stats()["rechecked"] >= 59 * 59
    M = 12
    lo, hi, r2, bins2, counts2 = cil.cil_pair_bins_adaptive(dev(A), dev(B), M)
    assert (lo, hi) == (D.min(), D.max())
    want_r = oracle_mod.radii_ladder(D.min(), D.max(), M)
    assert np.array_equal(r2, want_r)
    assert np.array_equal(bins2.cpu().numpy(), oracle_mod.bins_from_d2(D, want_r))
    assert np.array_equal(counts2, oracle_mod.counts_from_d2(D, want_r))


def test_adaptive_bins_rejects_a_degenerate_range(cil):
    A = np.ones((3, 8), dtype=np.float64)
    with pytest.raises(cil.CilError) as e:
        cil.cil_pair_bins_adaptive(dev(A), dev(A), 4)
    assert e.value.code == cil.CIL_EINVAL


@pytest.mark.parametrize("gather", [0, 1])
@pytest.mark.parametrize("M", [1, 13, 32, 33, 70])
def test_bootstrap_counts_bit_exact(cil, oracle_mod, M, gather):
    """Both bootstrap paths (matrix cores; gather) against the oracle, with
    ragged sizes (nA, nB not multiples of the tiles, n_boot = 50)."""
    A, B = sets(290, 75, 64, seed=M, dtype=np.float64)
    D = oracle_mod.pair_d2(A, B)
    radii = oracle_mod.radii_ladder(D.min(), D.max(), M)
    bins, _ = cil.cil_pair_bins(dev(A), dev(B), radii)
    ia, ib = cs.resample_halves(290, 75, 290, 75, 50, seed=M)
    want_c, want_y = oracle_mod.bootstrap_vectors(D, ia, ib, radii)
    cil.cil_set_option(cil.CIL_OPT_BOOTSTRAP_GATHER, gather)
    try:
        Yc, Y = cil.cil_bootstrap_features(bins, torch.from_numpy(ia), torch.from_numpy(ib), M)
    finally:
        cil.cil_set_option(cil.CIL_OPT_BOOTSTRAP_GATHER, 0)
    assert np.array_equal(Yc.cpu().numpy(), want_c)
    assert np.array_equal(Y.cpu().numpy(), want_y)


def test_bootstrap_high_multiplicity_falls_back_exactly(cil, oracle_mod):
    """A resample that repeats one pattern 300 times (not exact in bf16) still
    gives the oracle's counts (the gather path takes over)."""
    A, B = sets(40, 30, 16, seed=7, dtype=np.float64)
    D = oracle_mod.pair_d2(A, B)
    radii = oracle_mod.radii_ladder(D.min(), D.max(), 8)
    bins, _ = cil.cil_pair_bins(dev(A), dev(B), radii)
    ia = np.zeros((3, 400), dtype=np.int32)
    ia[:, 300:] = np.arange(100, dtype=np.int32)[None, :] % 40
    ib = np.tile(np.arange(30, dtype=np.int32), (3, 2))
    want_c, _ = oracle_mod.bootstrap_vectors(D, ia, ib, radii)
    Yc, _ = cil.cil_bootstrap_features(bins, torch.from_numpy(ia), torch.from_numpy(ib), 8)
    assert np.array_equal(Yc.cpu().numpy(), want_c)


def test_bootstrap_rejects_bad_index(cil):
    bins = torch.zeros((4, 4), dtype=torch.uint8, device="cuda")
    ia = torch.tensor([[0, 1, 9]], dtype=torch.int32)
    ib = torch.tensor([[0, 1]], dtype=torch.int32)
    with pytest.raises(cil.CilError) as e:
        cil.cil_bootstrap_features(bins, ia, ib, 3)
    assert e.value.code == cil.CIL_EINVAL


def test_loglik_matches_oracle(cil, oracle_mod):
    g = np.random.default_rng(12)
    P, n, M = 5, 200, 13
    Ys = []
    yo = []
    for p in range(P):
        Y = g.standard_normal((n, M)) @ g.standard_normal((M, M)) * 0.01 + 0.5
        if p == 1:
            Y[:, 0] = 1.0          # a constant bin, dropped
            Y[:, M - 1] = 0.0      # an empty bin, dropped
        Ys.append(Y)
        yo.append(Y.mean(0) + 0.01 * g.standard_normal(M))
    Ys = np.stack(Ys)
    yo = np.stack(yo)
    f, ll, me, stt = cil.cil_gaussian_loglik(dev(Ys), dev(yo))
    f, ll, me, stt = f.cpu().numpy(), ll.cpu().numpy(), me.cpu().numpy(), stt.cpu().numpy()
    for p in range(P):
        r = oracle_mod.gaussian_cost(Ys[p], yo[p])
        assert me[p] == r["m_eff"] and stt[p] == 0
        assert f[p] == pytest.approx(r["f"], rel=1e-10)
        assert ll[p] == pytest.approx(r["loglik"], rel=1e-10)


def test_loglik_not_spd(cil):
    g = np.random.default_rng(2)
    z = g.standard_normal(50)
    Y = np.stack([z, z, g.standard_normal(50)], 1)[None]          # two identical bins: singular
    f, ll, me, stt = cil.cil_gaussian_loglik(dev(Y), dev(np.zeros((1, 3))))
    assert int(stt.cpu()[0]) == cil.CIL_ENOTSPD and math.isnan(float(f.cpu()[0]))


def test_end_to_end_fhn32_plain_fp64(cil, oracle_mod):
    """FHN 32x32, 5000 fixed steps, two 64-pattern sets, 16 radii R0 1.2^-m:
    all 128 trajectories against the oracle's; then the statistic of the
    oracle's patterns on both sides (range, radii and counts bit-exact)."""
    w = cs.WORKLOADS["fhn32_fixed5000"]
    base = oracle_mod.homogeneous_state(w["model"], w["params"])
    sets_ = [cs.initial_conditions(base, w["n"], w["count"], seed=s, law=w["ic_law"]) for s in w["seeds"]]
    ics = np.concatenate(sets_)
    st = torch.tensor(ics, dtype=torch.float64, device="cuda")
    probs = cil.make_problems(w["n"], w["L"], w["nu"], w["params"], count=ics.shape[0])
    ref = ics.copy()
    done = 0
    # the trajectory error against the oracle, step count by step count: 1e-10
    # holds at 1000 steps; later, pattern selection amplifies the last-bit
    # differences of two correct algorithms (cosine transforms vs a banded
    # Cholesky solve) by orders of magnitude, so the 5000-step bar is looser
    for upto, bar in ((1000, 1e-10), (5000, 1e-8)):
        rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], upto - done, check_every=upto - done,
                                        path=cil.CIL_PATH_PLAIN)
        assert np.all(rep["status"] == 0)
        ref, _, _, _ = oracle_mod.imex_run(w["model"], w["params"], w["nu"], w["n"], w["L"], w["dt"], upto - done,
                                           0.0, upto - done, state=ref, nthreads=16)
        done = upto
        g = st.cpu().numpy()
        err = np.abs(g - ref).max() / np.abs(ref).max()
        print("fhn32 FP64 trajectory error at step %d: %.3e" % (upto, err), flush=True)
        assert err <= bar
    An, Bn = ref[:64].reshape(64, -1), ref[64:].reshape(64, -1)
    A = torch.tensor(An, device="cuda")
    B = torch.tensor(Bn, device="cuda")
    lo, hi = cil.cil_distance_range(A, B)
    D = oracle_mod.pair_d2(An, Bn)
    assert (lo, hi) == (D.min(), D.max())
    radii = oracle_mod.power_radii(math.sqrt(D.max()), w["radii_base"], w["M"])
    c, y = cil.cil_features(A, B, radii)
    assert np.array_equal(c, oracle_mod.counts_from_d2(D, radii))


def test_fhn32_fixed5000_fp32_statistic_within_two_percent(cil, oracle_mod):
    """The plain method's configuration on the batched FP32 path (fused
    stepper, the benchmark's batched leg): after 5000 FP32 steps the
    correlation integral vector of the 64 x 64 cross pairs under the oracle's
    16 radii R0 1.2^-m (eqs. eCDF, CIL) lies within 2 % (relative, Euclidean)
    of the oracle's vector from its FP64 trajectories."""
    w = cs.WORKLOADS["fhn32_fixed5000"]
    base = oracle_mod.homogeneous_state(w["model"], w["params"])
    ics = np.concatenate([cs.initial_conditions(base, w["n"], w["count"], seed=s, law=w["ic_law"])
                          for s in w["seeds"]])
    ics32 = ics.astype(np.float32).astype(np.float64)
    ref, _, _, _ = oracle_mod.imex_run(w["model"], w["params"], w["nu"], w["n"], w["L"], w["dt"], w["max_steps"],
                                       0.0, w["max_steps"], state=ics32.copy(), nthreads=16)
    An, Bn = ref[:64].reshape(64, -1), ref[64:].reshape(64, -1)
    D = oracle_mod.pair_d2(An, Bn)
    radii = oracle_mod.power_radii(math.sqrt(D.max()), w["radii_base"], w["M"])
    want = oracle_mod.counts_from_d2(D, radii) / float(D.size)
    st = torch.tensor(ics, dtype=torch.float32, device="cuda")
    probs = cil.make_problems(w["n"], w["L"], w["nu"], w["params"], count=ics.shape[0])
    rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], check_every=w["check_every"])
    assert np.all(rep["status"] == 0)
    P = st.reshape(128, -1)
    _, y = cil.cil_features(P[:64], P[64:], radii)
    rel = np.linalg.norm(y - want) / np.linalg.norm(want)
    print("fhn32 FP32 statistic: rel dev %.3e, counts %s vs %s" % (rel, (y * D.size).astype(int).tolist(),
                                                                   (want * D.size).astype(int).tolist()), flush=True)
    assert rel <= 0.02
