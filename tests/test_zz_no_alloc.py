"""The allocation-free bootstrap entry point (cil_bootstrap_features_noalloc)
against cil_bootstrap_features through the C ABI: identical resample counts
and vectors on two calls in a row (the second smaller, so the shared scratch
holds the first call's contents), on the matrix-core and the gather path,
and a clear error for sizes beyond the scratch maximum."""
import ctypes

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


def run(cil, fn, bins, ia, ib, M):
    nA, nB = bins.shape
    n_boot, kA = ia.shape
    kB = ib.shape[1]
    Yc = torch.full((n_boot, M), -1, dtype=torch.int64, device="cuda")
    Y = torch.full((n_boot, M), -1.0, dtype=torch.float64, device="cuda")
    rc = fn(ctypes.c_void_p(bins.data_ptr()), nA, nB, M, ctypes.c_void_p(ia.data_ptr()), kA,
            ctypes.c_void_p(ib.data_ptr()), kB, n_boot, ctypes.c_void_p(Yc.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, Yc.cpu().numpy(), Y.cpu().numpy()


def case(nA, nB, kA, kB, n_boot, M, seed):
    g = np.random.default_rng(seed)
    bins = torch.tensor(g.integers(0, M + 1, size=(nA, nB)), dtype=torch.uint8, device="cuda")
    ia = g.integers(0, nA, size=(n_boot, kA)).astype(np.int32)
    ib = g.integers(0, nB, size=(n_boot, kB)).astype(np.int32)
    return bins, torch.from_numpy(ia).cuda(), torch.from_numpy(ib).cuda()


@pytest.mark.parametrize("M", [13, 40])
def test_noalloc_matches_bootstrap_on_two_calls(cil, M):
    L = cil.lib()
    for nA, nB, kA, kB, n_boot, seed in ((300, 260, 300, 260, 200, 1), (40, 50, 30, 20, 17, 2)):
        bins, ia, ib = case(nA, nB, kA, kB, n_boot, M, seed)
        print("noalloc case M=%d nA=%d nB=%d kA=%d kB=%d n_boot=%d" % (M, nA, nB, kA, kB, n_boot), flush=True)
        rc0, c0, y0 = run(cil, L.cil_bootstrap_features, bins, ia, ib, M)
        rc1, c1, y1 = run(cil, L.cil_bootstrap_features_noalloc, bins, ia, ib, M)
        assert rc0 == 0 and rc1 == 0, (rc0, rc1, L.cil_last_error())
        assert np.array_equal(c0, c1)
        assert np.array_equal(y0, y1)
        # the resample vectors themselves, from the bins on the host
        b = bins.cpu().numpy()
        r = n_boot - 1
        sel = b[np.ix_(ia[r].cpu().numpy(), ib[r].cpu().numpy())]
        assert np.array_equal(c1[r], [(sel > m).sum() for m in range(M)])


def test_noalloc_resample_halves_workload_shape(cil):
    """The stationarity workload's bootstrap shape: halves of 250, 200
    resamples of the halves (Alg. 2bst), 13 radii."""
    L = cil.lib()
    g = np.random.default_rng(5)
    bins = torch.tensor(g.integers(0, 14, size=(250, 250)), dtype=torch.uint8, device="cuda")
    a, b = cs.resample_halves(250, 250, 250, 250, 200, seed=6)
    ia, ib = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    rc0, c0, y0 = run(cil, L.cil_bootstrap_features, bins, ia, ib, 13)
    rc1, c1, y1 = run(cil, L.cil_bootstrap_features_noalloc, bins, ia, ib, 13)
    assert rc0 == 0 and rc1 == 0
    assert np.array_equal(c0, c1) and np.array_equal(y0, y1)


def test_noalloc_rejects_sizes_beyond_its_scratch(cil):
    L = cil.lib()
    dummy = torch.zeros(16, dtype=torch.int32, device="cuda")
    out = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    rc = L.cil_bootstrap_features_noalloc(p, 8192, 8192, 13, p, 8192, p, 8192, 400, None,
                                          ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == cil.CIL_EINVAL
    assert b"scratch" in L.cil_last_error()
