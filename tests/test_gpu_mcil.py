"""Multi-feature CIL (Sec. 3.1) and min-max scaled data (Sec. 5) on the GPU
against the oracle: min-max scaling, derivative augmentation, per-segment
max-abs distances and their combinations, distance ranges and bins, all
bit-exact; W^{1,2} counts through the Gram path on augmented vectors,
bit-exact; the sum-of-L2 W^{1,2} variant from per-part canonical squared
distances, bit-exact; the concatenated six-norm bootstrap vectors bit-exact
and their likelihood within 1e-10.
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_minmax_scale_bit_exact(cil, oracle_mod, dtype):
    g = np.random.default_rng(1)
    x = (3.0 + g.standard_normal((7, 2, 33, 33)) * 10.0 ** g.integers(-3, 3, size=(7, 2, 1, 1))).astype(dtype)
    x[2, 1] = 4.5                                   # a constant species
    got = cil.cil_minmax_scale(dev(x), 33).cpu().numpy()
    assert np.array_equal(got, oracle_mod.minmax_scale(x))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [2, 17, 64])
def test_augment_bit_exact(cil, oracle_mod, dtype, n):
    g = np.random.default_rng(n)
    x = g.standard_normal((5, 2, n, n)).astype(dtype)
    got = cil.cil_augment_patterns(dev(x), n, 7.5).cpu().numpy()
    assert got.shape == (5, cil.augmented_dim(n))
    assert np.array_equal(got, oracle_mod.augment(x, n, 7.5))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("nA,nB,ends", [(1, 1, [5]), (70, 131, [100, 100, 333, 340]), (64, 64, [2048]),
                                        (129, 65, [17, 600, 1000])])
def test_pair_maxabs_bit_exact(cil, oracle_mod, dtype, nA, nB, ends):
    g = np.random.default_rng(nA + nB)
    d = ends[-1]
    A = (g.standard_normal((nA, d)) * 10.0 ** g.integers(-4, 4, size=(nA, d))).astype(dtype)
    B = (g.standard_normal((nB, d)) * 10.0 ** g.integers(-4, 4, size=(nB, d))).astype(dtype)
    D = cil.cil_pair_maxabs(dev(A), dev(B), ends)
    want = oracle_mod.pair_maxabs(A, B, ends)
    assert np.array_equal(D.cpu().numpy(), want)
    for mode in (0, 1, 2):
        assert np.array_equal(cil.cil_combine_segments(D, mode).cpu().numpy(), oracle_mod.combine_segments(want, mode))


def test_value_range_and_bins_bit_exact(cil, oracle_mod):
    g = np.random.default_rng(9)
    V = g.random((300, 257)) * 5.0
    V[3, 4] = 0.125
    lo, hi = cil.cil_value_range(dev(V))
    assert (lo, hi) == (V.min(), V.max())
    radii = oracle_mod.radii_ladder(lo * lo, hi * hi, 20)
    radii[5] = V[10, 10]                            # a tie: strict comparison
    radii = np.sort(radii)[::-1].copy()
    bins, counts = cil.cil_bin_values(dev(V), radii)
    assert np.array_equal(bins.cpu().numpy(), oracle_mod.bins_from_values(V, radii))
    assert np.array_equal(counts, oracle_mod.counts_from_values(V, radii))


def test_feature_argument_errors(cil):
    x = torch.zeros(2, 2, 4, 4, device="cuda")
    with pytest.raises(cil.CilError):
        cil.cil_augment_patterns(x, 1, 1.0)
    with pytest.raises(cil.CilError):
        cil.cil_pair_maxabs(x.reshape(2, -1), x.reshape(2, -1), [20, 10])
    with pytest.raises(cil.CilError):
        cil.cil_pair_maxabs(x.reshape(2, -1), x.reshape(2, -1), [40])
    with pytest.raises(cil.CilError):
        cil.cil_bin_values(torch.zeros(4, dtype=torch.float64, device="cuda"), [1.0, 2.0])


def mcil_features(cil, P, n, L, M, ia, ib):
    """Six-norm bootstrap vectors on the GPU: L2, L-inf, W^{1,2}, W^{1,inf}, its
    sum variant and the sum-of-L2 W^{1,2} variant, each with its own adaptive
    radii (Sec. 3.2)."""
    half = P.shape[0] // 2
    nn2 = 2 * n * n
    ne2 = 2 * n * (n - 1)
    Aug = cil.cil_augment_patterns(P, n, L)
    Ys, radii_all = [], []
    tA, tB = torch.from_numpy(ia), torch.from_numpy(ib)
    # per-part canonical squared distances of all pairs, for the sum-of-L2 variant
    ii = torch.arange(half, device="cuda").repeat_interleave(half)
    jj = torch.arange(half, device="cuda").repeat(half)
    parts = []
    for a, b in ((0, nn2), (nn2, nn2 + ne2), (nn2 + ne2, nn2 + 2 * ne2)):
        Xs = Aug[:, a:b].contiguous()
        parts.append(cil.cil_canonical_d2(Xs[:half], Xs[half:], ii, jj).reshape(half, half))
    Wsum = cil.cil_combine_segments(torch.stack(parts, dim=-1).contiguous(), 2)
    # L2 and W^{1,2}: squared distances through the counting path
    for X in (P.reshape(P.shape[0], -1), Aug):
        _, _, radii, bins, _ = cil.cil_pair_bins_adaptive(X[:half], X[half:], M)
        _, Y = cil.cil_bootstrap_features(bins, tA, tB, M)
        Ys.append(Y)
        radii_all.append(radii)
    # the max-abs family from per-segment maxima of the augmented vectors
    D = cil.cil_pair_maxabs(Aug[:half], Aug[half:], [nn2, nn2 + ne2, nn2 + 2 * ne2])
    for V in (D[..., 0].contiguous(), cil.cil_combine_segments(D, 0), cil.cil_combine_segments(D, 1), Wsum):
        lo, hi = cil.cil_value_range(V)
        radii = cil.cil_radii(lo * lo, hi * hi, M)
        bins, _ = cil.cil_bin_values(V, radii)
        _, Y = cil.cil_bootstrap_features(bins, tA, tB, M)
        Ys.append(Y)
        radii_all.append(radii)
    return torch.cat(Ys, dim=1).contiguous(), radii_all


def oracle_mcil(o, Pn, n, L, M, ia, ib):
    half = Pn.shape[0] // 2
    nn2 = 2 * n * n
    ne2 = 2 * n * (n - 1)
    Aug = o.augment(Pn, n, L)
    Ys, radii_all = [], []
    for X in (Pn.reshape(Pn.shape[0], -1), Aug):
        D = o.pair_d2(X[:half], X[half:], nthreads=8)
        radii = o.radii_ladder(D.min(), D.max(), M)
        _, Y = o.bootstrap_vectors(D, ia, ib, radii, nthreads=8)
        Ys.append(Y)
        radii_all.append(radii)
    Dm = o.pair_maxabs(Aug[:half], Aug[half:], [nn2, nn2 + ne2, nn2 + 2 * ne2])
    parts = np.stack([o.pair_d2(Aug[:half, a:b], Aug[half:, a:b], nthreads=8)
                      for a, b in ((0, nn2), (nn2, nn2 + ne2), (nn2 + ne2, nn2 + 2 * ne2))], axis=-1)
    for V in (Dm[..., 0], o.combine_segments(Dm, 0), o.combine_segments(Dm, 1), o.combine_segments(parts, 2)):
        radii = o.radii_ladder(V.min() ** 2, V.max() ** 2, M)
        # bootstrap on distances: the squared values keep the order and the
        # radii ladder's squares decide the same bins
        b = o.bins_from_values(V, radii)
        Yc = np.zeros((ia.shape[0], M), dtype=np.int64)
        for r in range(ia.shape[0]):
            sub = b[np.ix_(ia[r], ib[r])]
            Yc[r] = [(sub >= m + 1).sum() for m in range(M)]
        Ys.append(Yc / float(ia.shape[1] * ib.shape[1]))
        radii_all.append(radii)
    return np.concatenate(Ys, axis=1), radii_all


@pytest.mark.parametrize("scaled", [False, True])
def test_multi_feature_vectors_and_likelihood(cil, oracle_mod, scaled):
    n, L, M, count, n_boot = 32, 1.0, 10, 64, 60
    P = cs.stripe_patterns(count, n, seed=21).astype(np.float32)
    if scaled:
        P = oracle_mod.minmax_scale(P)
    Pd = dev(P)
    if scaled:                                      # the GPU scales its own copy of the same input
        Pd = cil.cil_minmax_scale(dev(cs.stripe_patterns(count, n, seed=21).astype(np.float32)), n)
        assert np.array_equal(Pd.cpu().numpy(), P)
    half = count // 2
    ia, ib = cs.resample_halves(half, half, half, half, n_boot, seed=22)
    Y, radii = mcil_features(cil, Pd, n, L, M, ia, ib)
    want, wradii = oracle_mcil(oracle_mod, P, n, L, M, ia, ib)
    for r, w in zip(radii, wradii):
        assert np.array_equal(r, w)
    assert np.array_equal(Y.cpu().numpy(), want)
    y_obs = want[0]
    f, ll, me, st = cil.cil_gaussian_loglik(Y, torch.tensor(y_obs, dtype=torch.float64, device="cuda"))
    ref = oracle_mod.gaussian_cost(want, y_obs)
    assert int(me.cpu()[0]) == ref["m_eff"]
    if ref["ok"]:
        assert float(f.cpu()[0]) == pytest.approx(ref["f"], rel=1e-10)
        assert float(ll.cpu()[0]) == pytest.approx(ref["loglik"], rel=1e-10)
    print("MCIL (scaled=%s): %d features, m_eff %d" % (scaled, Y.shape[1], ref["m_eff"]))
