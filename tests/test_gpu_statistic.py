"""The synthetic-likelihood statistic in one call (cil_statistic_adaptive,
Alg. 2bst) against the same steps as separate calls and against the oracle.

Integers (bins, counts, bootstrap vectors' counts) and the values formed from
them are bit-exact; the likelihood equals the separate call's bit for bit and
is held to the oracle within 1e-10 relative.
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def same_bits(a, b):
    """Equal bit for bit (NaN included)."""
    if a.dtype == torch.float64:
        a, b = a.view(torch.int64), b.view(torch.int64)
    return torch.equal(a, b)


def separate(cil, A, B, M, ia, ib, law):
    lo, hi, radii, bins, counts = cil.cil_pair_bins_adaptive(A, B, M, law=law)
    _, Y = cil.cil_bootstrap_features(bins, ia, ib, M, want_counts=False)
    y_obs = torch.from_numpy(counts / float(A.shape[0] * B.shape[0])).cuda()
    out = cil.cil_gaussian_loglik(Y, y_obs)
    return lo, hi, radii, counts, bins, Y, y_obs, out


def check_same(cil, oracle_mod, A, B, M, n_boot, law, seed):
    nA, nB = A.shape[0], B.shape[0]
    ia, ib = cs.resample_halves(nA, nB, nA, nB, n_boot, seed=seed)
    tia, tib = torch.from_numpy(ia), torch.from_numpy(ib)
    dA, dB = dev(A), dev(B)
    want = separate(cil, dA, dB, M, tia, tib, law)
    got = cil.cil_statistic_adaptive(dA, dB, M, tia, tib, law=law)
    assert (got[0], got[1]) == (want[0], want[1])
    assert np.array_equal(got[2], want[2])
    assert np.array_equal(got[3], want[3])
    assert same_bits(got[4], want[4])
    assert same_bits(got[5], want[5])
    assert same_bits(got[6], want[6])
    for g, w in zip(got[7], want[7]):
        assert same_bits(g, w)
    # and the oracle: range, radii, counts, bins, bootstrap vectors, likelihood
    D = oracle_mod.pair_d2(A, B)
    assert (got[0], got[1]) == (D.min(), D.max())
    r = oracle_mod.radii_ladder(D.min(), D.max(), M, law="power" if law == 0 else "linear")
    assert np.array_equal(got[2], r)
    assert np.array_equal(got[3], oracle_mod.counts_from_d2(D, r))
    assert np.array_equal(got[4].cpu().numpy(), oracle_mod.bins_from_d2(D, r))
    _, want_y = oracle_mod.bootstrap_vectors(D, ia, ib, r)
    assert np.array_equal(got[5].cpu().numpy(), want_y)
    y_obs = oracle_mod.counts_from_d2(D, r) / float(nA * nB)
    assert np.array_equal(got[6].cpu().numpy(), y_obs)
    c = oracle_mod.gaussian_cost(want_y, y_obs)
    f, ll, me, stt = (t.cpu().numpy()[0] for t in got[7])
    if c["ok"]:
        assert stt == 0 and me == c["m_eff"]
        assert f == pytest.approx(c["f"], rel=1e-10)
        assert ll == pytest.approx(c["loglik"], rel=1e-10)
    else:
        assert stt == cil.CIL_ENOTSPD
    return got


@pytest.fixture(params=[1, 0, 2], ids=["device_radii", "host_radii", "forced_second_pass"])
def radii_mode(cil, request):
    """The radii formed on the device and checked (the default), formed on the
    host, or the device's check forced to fail so that the call redoes the
    statistic with the host's radii."""
    cil.cil_set_option(cil.CIL_OPT_STAT_DEVICE_RADII, request.param)
    yield request.param
    cil.cil_set_option(cil.CIL_OPT_STAT_DEVICE_RADII, 1)


@pytest.mark.parametrize("dtype,nA,nB,d,M,n_boot,law", [
    (np.float32, 250, 250, 8192, 13, 200, 0),      # the shape of the benchmarked statistic
    (np.float64, 70, 90, 515, 16, 50, 1),
    (np.float32, 37, 61, 200, 5, 9, 0),
    (np.float64, 1, 300, 64, 7, 2, 0),
    (np.float32, 120, 140, 4096, 64, 20, 1),
])
def test_statistic_matches_separate_calls_and_oracle(cil, oracle_mod, radii_mode, dtype, nA, nB, d, M, n_boot, law):
    g = np.random.default_rng(nA + d)
    A = (0.3 * g.standard_normal((nA, d)) + 1.0).astype(dtype)
    B = (0.3 * g.standard_normal((nB, d)) + 1.0).astype(dtype)
    check_same(cil, oracle_mod, A, B, M, n_boot, law, seed=M)


def radius_heavy_sets(dtype, d=515, copies=60, M=6):
    """Sets whose (copies - 1)^2 cross pairs of copies all lie at the first
    radius of the adaptive ladder (to FP rounding): A = [P e1; 0 ...],
    B = [Q e0; t e0 ...] (plus a common offset in FP32, so that the fast
    pass's bound is not zero), so the pair distances are t (the copies), Q
    (the smallest), sqrt(P^2 + t^2) (the largest) and P; P is solved for so
    that R_1 = R_0 (R_0 / R_M)^(-1/M) equals t."""
    t, Q = 3.0, 1.0
    lo_p, hi_p = 1.0, 1e4
    for _ in range(200):
        P = 0.5 * (lo_p + hi_p)
        R0 = math.sqrt(P * P + t * t)
        R1 = R0 * (R0 / Q) ** (-1.0 / M)
        if R1 < t:
            lo_p = P
        else:
            hi_p = P
    A = np.zeros((copies, d), dtype=dtype)
    B = np.zeros((copies, d), dtype=dtype)
    A[0, 1] = P
    B[0, 0] = Q
    B[1:, 0] = t
    if dtype == np.float32:
        off = np.random.default_rng(4).uniform(0.5, 1.5, d)
        A = (A + off).astype(dtype)
        B = (B + off).astype(dtype)
    return A, B, M


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_statistic_with_a_long_recheck_list(cil, oracle_mod, radii_mode, dtype):
    """3481 pairs on a radius: longer than the first canonical launch covers,
    so the strided launch after it finishes the list on the device (the call
    does not read the list's length in between); bins and counts stay the
    oracle's."""
    A, B, M = radius_heavy_sets(dtype)
    check_same(cil, oracle_mod, A, B, M, n_boot=20, law=0, seed=3)
    assert cil.cil_last_distance_stats()["rechecked"] >= 59 * 59


def test_statistic_twice_smaller_second(cil, oracle_mod):
    """Two calls in a row, the second on smaller sets (the workspaces and
    staging are reused)."""
    g = np.random.default_rng(5)
    A = g.standard_normal((120, 300)).astype(np.float32)
    B = g.standard_normal((80, 300)).astype(np.float32)
    check_same(cil, oracle_mod, A, B, 10, 30, 0, seed=1)
    check_same(cil, oracle_mod, A[:17], B[:23], 4, 5, 0, seed=2)


def test_statistic_rejects_bad_bootstrap_index(cil, radii_mode):
    g = np.random.default_rng(6)
    A = dev(g.standard_normal((4, 16)))
    B = dev(g.standard_normal((5, 16)))
    ia = torch.tensor([[0, 1, 9]] * 2, dtype=torch.int32)
    ib = torch.tensor([[0, 1]] * 2, dtype=torch.int32)
    with pytest.raises(cil.CilError) as e:
        cil.cil_statistic_adaptive(A, B, 3, ia, ib)
    assert e.value.code == cil.CIL_EINVAL
    # the library stays usable
    ia = torch.tensor([[0, 1, 3]] * 2, dtype=torch.int32)
    cil.cil_statistic_adaptive(A, B, 3, ia, ib)


def test_statistic_rejects_bad_sizes(cil, radii_mode):
    A = dev(np.ones((3, 8)))
    ia = torch.zeros((2, 3), dtype=torch.int32)
    with pytest.raises(cil.CilError):
        cil.cil_statistic_adaptive(A, A, 65, ia, ia)          # M > 64
    with pytest.raises(cil.CilError):
        cil.cil_statistic_adaptive(A, A, 3, ia[:1], ia[:1])   # n_boot < 2
    with pytest.raises(cil.CilError) as e:
        cil.cil_statistic_adaptive(A, A, 3, ia, ia)           # every distance 0: degenerate range
    assert e.value.code == cil.CIL_EINVAL


def test_statistic_radii_across_many_ranges(cil):
    """Over 200 random ranges, both laws and M up to 64, the call's radii are
    the host's ladder (cil_radii, the oracle's expression), whether the
    device's ladder agreed or the call took its second pass."""
    g = np.random.default_rng(11)
    ia = torch.zeros((2, 3), dtype=torch.int32)
    calls = 200
    cil.cil_profile(1)
    try:
        for t in range(calls):
            d = 1 + int(g.integers(1, 40))
            A = dev(g.standard_normal((3, d)) * float(np.exp(g.uniform(-3, 3))))
            B = dev(g.standard_normal((3, d)) * float(np.exp(g.uniform(-3, 3))) + float(g.uniform(-2, 2)))
            M = int(g.integers(1, 65))
            law = int(t % 2)
            lo, hi, radii, counts, *_ = cil.cil_statistic_adaptive(A, B, M, ia, ia, law=law)
            assert np.array_equal(radii, cil.cil_radii(lo, hi, M, law=law))
        passes = cil.cil_profile_read("k_classify_range1")[0]      # one range pass per call, two after a mismatch
    finally:
        cil.cil_profile(0)
    assert calls <= passes <= calls + calls // 10


def _cr_pow(x, y):
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    return float(str((Decimal(x).ln() * Decimal(y)).exp()))


def _ladders_differ(lo, hi, M):
    """Whether the device's ladder (correctly rounded powers) differs from
    the host's (the C library's pow) for this range."""
    R0, RM = math.sqrt(hi), math.sqrt(lo)
    bh, bd = math.pow(R0 / RM, 1.0 / M), _cr_pow(R0 / RM, 1.0 / M)
    return any(R0 * math.pow(bh, -m) != R0 * _cr_pow(bd, -m) for m in range(1, M + 1))


def _range_passes(cil, A, B, M, ia, ib):
    cil.cil_profile(1)
    try:
        got = cil.cil_statistic_adaptive(A, B, M, ia, ib)
        return got, cil.cil_profile_read("k_classify_range1")[0]
    finally:
        cil.cil_profile(0)


@pytest.mark.parametrize("near_pair", [False, True])
def test_statistic_when_the_ladders_differ(cil, oracle_mod, near_pair):
    """1-D sets with squared distances 56^2 .. 206^2 and M = 9: there the C
    library's pow misrounds b^-6, and R_6 = R_0 b^-6 with it, by one unit, so
    the device's ladder differs from the host's.  With no pair near a
    threshold the bins stand and the call makes one pass; with a pair at R_6
    (from the host's ladder) it makes a second pass with the host's radii.
    Either way the results are the separate calls' and the oracle's."""
    M = 9
    A = np.zeros((1, 1))
    B = np.array([[56.0], [206.0], [80.0], [120.0], [170.0]])
    r = cil.cil_radii(56.0 ** 2, 206.0 ** 2, M)
    if near_pair:
        B = np.vstack([B, [[r[5]]]])
    differ = _ladders_differ(56.0 ** 2, 206.0 ** 2, M)
    assert differ
    ia, ib = cs.resample_halves(1, B.shape[0], 1, B.shape[0], 6, seed=4)
    _, passes = _range_passes(cil, dev(A), dev(B), M, torch.from_numpy(ia), torch.from_numpy(ib))
    assert passes == (2 if (differ and near_pair) else 1)
    check_same(cil, oracle_mod, A, B, M, 6, 0, seed=4)
