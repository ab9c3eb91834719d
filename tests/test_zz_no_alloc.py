"""kmeans_assign_static: the assignment pass that allocates nothing (its
workspace is a fixed per-device array) returns bitwise what kmeans_assign
returns, on two calls in a row (the second smaller, so stale contents of the
array from the first must not leak), and rejects a pass whose workspace
would not fit the array."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
km = pytest.importorskip("paper_2407_12208_amd")


@pytest.fixture(scope="module")
def ctx():
    c = km.Context(0)
    yield c
    c.close()


def run_both(ctx, X, C, prec, hint=None):
    out = []
    for static in (False, True):
        lab = hint.clone() if hint is not None else None
        labels, mind, sse, st = km.kmeans_assign(ctx, X, C, prec, labels=lab, mindist=True,
                                                 sse=True, stats=True,
                                                 labels_hint=hint is not None, static=static)
        torch.cuda.synchronize()
        out.append((labels.cpu().numpy(), mind.cpu().numpy(), float(sse.cpu()[0]), st))
    return out


@pytest.mark.parametrize("low", [km.KM_LOW_FP16, km.KM_LOW_BF16])
def test_static_equals_assign_two_calls(ctx, low):
    prec = km.Precision(low, km.KM_ALPHA_PAPER_EQ if low == km.KM_LOW_FP16 else km.KM_ALPHA_HW, 5.0)
    # first call: matrix-core kernel (d = 64, k = 300); second, smaller:
    # the small-problem kernel (d = 16, k = 40)
    for (n, d, k, seed) in ((40_000, 64, 300, 31), (9_000, 16, 40, 32)):
        Xh, _, _ = W.blobs(n, d, k, seed)
        Ch = W.init_centroids(Xh, k, seed + 100)
        X = torch.from_numpy(Xh).cuda()
        C = torch.from_numpy(Ch).cuda()
        (l0, m0, s0, st0), (l1, m1, s1, st1) = run_both(ctx, X, C, prec)
        assert np.array_equal(l0, l1)
        assert np.array_equal(m0.view(np.uint32), m1.view(np.uint32))
        assert s0 == s1
        assert st0["n_corrected"] == st1["n_corrected"] and st0["n_pairs"] == st1["n_pairs"]
        assert st0["data_status"] == st1["data_status"] == 0
        # with the labels as a seed (a Lloyd round): the same outputs again
        hint = torch.from_numpy(l0).cuda()
        (l2, m2, s2, _), (l3, m3, s3, _) = run_both(ctx, X, C, prec, hint=hint)
        assert np.array_equal(l2, l0) and np.array_equal(l3, l0)
        assert s2 == s0 and s3 == s0


def test_static_fp64_direct_route(ctx):
    Xh, _, _ = W.blobs(5_000, 24, 20, 33)
    Ch = W.init_centroids(Xh, 20, 133)
    X = torch.from_numpy(Xh).cuda()
    C = torch.from_numpy(Ch).cuda()
    (l0, m0, s0, _), (l1, m1, s1, _) = run_both(ctx, X, C, km.Precision(km.KM_EXACT64))
    assert np.array_equal(l0, l1) and np.array_equal(m0, m1) and s0 == s1


def test_static_rejects_oversized_workspace(ctx):
    # quantised centres alone: 65,536 x 256 x 4 bytes = 64 MiB > the array
    k, d = 65536, 256
    C = torch.zeros((k, d), dtype=torch.float32, device="cuda")
    X = torch.zeros((k, d), dtype=torch.float32, device="cuda")
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign_static(ctx, X, C, km.Precision(km.KM_LOW_FP16))
    assert e.value.code == -8  # KM_ERR_UNSUPPORTED
