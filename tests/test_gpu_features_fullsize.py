"""Full-size checks of the CIL statistic alone on 4096 FP32 stand-in patterns of
dimension 32768 (two halves of 2048, 4 194 304 cross pairs, 32 power-law
radii, 200 bootstrap resamples): the launch configuration of
`bench.py --workload features4096`.

The oracle cannot take all 4.2e6 canonical distances at d = 32768 in seconds,
so it checks: the range end points (the oracle's canonical distance of the
candidate pairs an FP64 Gram ranks first) and the radii built from them; the
bins of 3000 random pairs and of every pair whose distance lies within 1e-4
(relative) of a radius, bit-exact against the oracle's bins of its own
canonical distances under its own radii; counts and bootstrap vectors through
properties that hold at any size (histogram of the bins, monotonicity, the
identity resample).  The FP64 Gram only selects which pairs to check: no GPU
value enters the oracle.
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


@pytest.fixture(scope="module")
def feat(cil, oracle_mod):
    w = cs.WORKLOADS["features4096"]
    count, n, M = w["count"], w["n"], w["M"]
    half, d = count // 2, 2 * n * n
    print("features4096: generating patterns", flush=True)
    host = cs.stripe_patterns(count, n, seed=w["seeds"][0]).reshape(count, d)
    pats = torch.from_numpy(host).cuda()
    A, Bs = pats[:half], pats[half:]
    print("features4096: range, radii, bins", flush=True)
    lo, hi, radii, bins, counts = cil.cil_pair_bins_adaptive(A, Bs, M)     # as the benchmark runs it
    torch.cuda.synchronize()
    # FP64 Gram distances, only to rank candidate pairs for the oracle
    A64, B64 = A.double(), Bs.double()
    D64 = ((A64 * A64).sum(1)[:, None] + (B64 * B64).sum(1)[None, :] - 2.0 * (A64 @ B64.T)).cpu().numpy()
    # the oracle's range: canonical distances of the 16 smallest and 16 largest
    # candidates, and its radii from them (no GPU result enters the oracle)
    flat = D64.ravel()
    ends = []
    for idx in (np.argsort(flat)[:16], np.argsort(flat)[-16:]):
        ends.append(oracle_mod.pair_d2_sampled(host[:half], host[half:], idx // half, idx % half, nthreads=8))
    o_lo, o_hi = ends[0].min(), ends[1].max()
    o_radii = oracle_mod.radii_ladder(o_lo, o_hi, M)
    return dict(w=w, host=host, half=half, A=A, Bs=Bs, lo=lo, hi=hi, radii=radii, bins=bins, counts=counts, D64=D64,
                o_lo=o_lo, o_hi=o_hi, o_radii=o_radii)


def test_range_end_points(cil, oracle_mod, feat):
    assert (feat["lo"], feat["hi"]) == (feat["o_lo"], feat["o_hi"])
    assert np.array_equal(feat["radii"], feat["o_radii"])
    assert cil.cil_distance_range(feat["A"], feat["Bs"]) == (feat["lo"], feat["hi"])


def test_bins_on_random_and_near_radius_pairs(cil, oracle_mod, feat):
    """Sec. 2.1 eq. (eCDF): bin of a pair = #{m : D < R_m^2}, strict; the
    oracle takes its canonical D of each checked pair and its own radii."""
    host, half, D64, o_radii = feat["host"], feat["half"], feat["D64"], feat["o_radii"]
    g = np.random.default_rng(11)
    rand = g.integers(0, half * half, size=3000)
    flat = D64.ravel()
    near = np.zeros(flat.size, dtype=bool)
    for t in o_radii * o_radii:
        near |= np.abs(flat - t) <= 1e-4 * t
    near_idx = np.flatnonzero(near)
    idx = np.concatenate([rand, near_idx])
    ia, jb = idx // half, idx % half
    print("features4096: oracle distances of %d random + %d near-radius pairs" % (rand.size, near_idx.size),
          flush=True)
    Dc = oracle_mod.pair_d2_sampled(host[:half], host[half:], ia, jb, nthreads=16)
    want = oracle_mod.bins_from_d2(Dc, o_radii)
    got = feat["bins"].cpu().numpy()[ia, jb]
    assert near_idx.size > 0
    assert np.array_equal(got, want)


def test_counts_are_the_bin_histogram(cil, feat):
    M = feat["w"]["M"]
    h = torch.bincount(feat["bins"].reshape(-1).long(), minlength=M + 1).cpu().numpy()
    tail = np.cumsum(h[::-1])[::-1]           # pairs with bin >= m
    assert np.array_equal(feat["counts"], tail[1:M + 1])
    assert np.all(np.diff(feat["counts"]) <= 0)
    assert feat["counts"][0] <= feat["half"] ** 2


def test_bootstrap_properties(cil, feat):
    w, half, M = feat["w"], feat["half"], feat["w"]["M"]
    ia, ib = cs.resample_halves(half, half, half, half, w["n_boot"], seed=w["boot_seed"])
    ia[0] = np.arange(half, dtype=np.int32)
    ib[0] = np.arange(half, dtype=np.int32)
    Yc, Y = cil.cil_bootstrap_features(feat["bins"], torch.from_numpy(ia), torch.from_numpy(ib), M)
    Yc, Y = Yc.cpu().numpy(), Y.cpu().numpy()
    assert np.array_equal(Yc[0], feat["counts"])                 # identity resample = full vector
    assert np.all(np.diff(Yc, axis=1) <= 0) and np.all(Yc >= 0) and np.all(Yc <= half * half)
    assert np.array_equal(Y, Yc / float(half * half))
