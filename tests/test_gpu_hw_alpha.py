"""GPU parity of the hardware-aware reliability threshold (KM_ALPHA_HW: the
error decomposition of Section 4.3 with the cross term accumulated in FP32
by the matrix cores) against the CPU oracle, through the C ABI: the large
and the small-problem assignment kernels, and a Lloyd solve."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import check_assignment

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
km = pytest.importorskip("paper_2407_12208_amd")


@pytest.fixture(scope="module")
def ctx():
    c = km.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def hw(low):
    return km.Precision(low, km.KM_ALPHA_HW, 5.0, 0.0)


@pytest.mark.parametrize("low,fmt", [(km.KM_LOW_FP16, 0), (km.KM_LOW_BF16, 1)])
@pytest.mark.parametrize("d,k", [(64, 100), (128, 300), (5, 40), (24, 64), (200, 50)])
def test_hw_alpha_assign_parity(ctx, low, fmt, d, k):
    # blobs with per-blob spread log-uniform in [0.1, 2] around centres in
    # [-50, 50]^d: the large-clustering workload's structure at test size
    n = 3000 + d
    X, _, _ = W.blobs(n, d, k, seed=900 + d + k, center_box=(-50, 50), std_range=(0.1, 2.0))
    C = W.init_centroids(X, k, 901 + d)
    labels, mind, sse, st = km.kmeans_assign(ctx, dev(X), dev(C), hw(low), mindist=True,
                                             sse=True, stats=True)
    a_ref = oracle.alpha_value(fmt, d, 5.0, "hw")
    assert abs(st["alpha_used"] - a_ref) <= 1e-6 * a_ref  # applied as FP32
    assert st["data_status"] == 0
    check_assignment(X, C, fmt, st["alpha_used"], host(labels), host(mind), float(host(sse)[0]),
                     st["n_corrected"], min_coverage=0.9)
    if low == km.KM_LOW_BF16 and d >= 64:
        # the paper's alpha flags every pair here; this one a small fraction
        assert st["n_corrected"] < 0.05 * n * k


def test_hw_alpha_bf16_lloyd(ctx):
    # BF16 Lloyd solve on large-clustering-shaped data: the final pass obeys
    # the parity contract against the final centres, the SSE history never
    # increases beyond rounding, and few pairs are corrected
    n, d, k = 20000, 64, 64
    X, _, _ = W.blobs(n, d, k, seed=910, center_box=(-50, 50), std_range=(0.1, 2.0))
    C = dev(W.init_centroids(X, k, 911))
    C, labels, mind, hist, st = km.kmeans_lloyd(ctx, dev(X), C, 10, prec=hw(km.KM_LOW_BF16),
                                                mindist=True, sse_hist=True, stats=True, sync=True)
    h = host(hist)
    assert np.all(np.diff(h) <= 1e-6 * h[:-1])
    assert st["n_corrected"] < 0.05 * n * k * 11
    check_assignment(X, host(C), 1, st["alpha_used"], host(labels), host(mind), float(h[-1]), None,
                     min_coverage=0.9)
