"""GPU parity of the assignment pass on small problems (d <= 32, k <= 64),
the shapes served by the kernel whose centres stay in registers: every
boundary of its row capacity (8 / 16 / 32 coordinates) and of its centre
blocks (32 / 64 centres), ragged point counts, the launch tiers that sweep
one, two and four groups of points per wave, unaligned rows, uniform low
precision, dense flags and the per-pair statistics, against the CPU oracle
through the C ABI."""

import numpy as np
import pytest

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


def prec(low=km.KM_LOW_FP16, mode=km.KM_ALPHA_PAPER_EQ):
    return km.Precision(low, mode, 5.0, 0.0)


def _assign(ctx, Xd, Cd, p):
    labels, mind, sse, st = km.kmeans_assign(ctx, Xd, Cd, p, mindist=True, sse=True, stats=True)
    return host(labels), host(mind), float(host(sse)[0]), st


@pytest.mark.parametrize("low,fmt", [(km.KM_LOW_FP16, 0), (km.KM_LOW_BF16, 1)])
@pytest.mark.parametrize("d,k", [(1, 5), (4, 32), (5, 33), (8, 64), (9, 1), (16, 31),
                                 (17, 64), (31, 2), (32, 48), (3, 64)])
def test_small_shapes(ctx, low, fmt, d, k):
    n = 2000 + 37 * d + k  # ragged: not a multiple of the 128 points of a workgroup
    X, _, _ = W.blobs(n, d, k, seed=700 + 31 * d + k, std=0.5)
    C = W.init_centroids(X, k, 701 + d)
    labels, mind, sse, st = _assign(ctx, dev(X), dev(C), prec(low))
    assert st["data_status"] == 0
    assert st["n_pairs"] == n * k
    check_assignment(X, C, fmt, st["alpha_used"], labels, mind, sse, st["n_corrected"],
                     min_coverage=0.9)


@pytest.mark.parametrize("n", [1_100_000, 2_200_000, 4_300_000])
def test_small_launch_tiers_sampled(ctx, n):
    # 2, 4 and 8 groups of 32 points per wave; sampled rows against the oracle,
    # the SSE against the oracle's sum over the GPU's labels
    d, k = 5, 40
    X, _, _ = W.blobs(n, d, k, seed=n, std=0.3)
    C = W.init_centroids(X, k, 5)
    labels, mind, sse, st = _assign(ctx, dev(X), dev(C), prec())
    assert st["data_status"] == 0
    g = np.random.default_rng(n)
    rows = np.unique(np.concatenate([g.choice(n, 20000, replace=False), np.arange(n - 300, n)]))
    check_assignment(X, C, 0, st["alpha_used"], labels, mind, None, None, rows=rows,
                     min_coverage=0.95)
    assert np.all((labels >= 0) & (labels < k))
    assert abs(sse - float(np.sum(mind.astype(np.float64)))) <= 1e-5 * sse


def test_small_unaligned_rows(ctx):
    # d = 8 with the point array starting 4 bytes into its allocation: the
    # row loads cannot use 16-byte accesses
    n, d, k = 3001, 8, 20
    X, _, _ = W.blobs(n, d, k, seed=88, std=0.4)
    C = W.init_centroids(X, k, 89)
    buf = torch.zeros(n * d + 1, dtype=torch.float32, device="cuda")
    buf[1:] = dev(X.reshape(-1))
    Xd = buf[1:].view(n, d)
    assert Xd.data_ptr() % 16 != 0
    labels, mind, sse, st = _assign(ctx, Xd, dev(C), prec())
    check_assignment(X, C, 0, st["alpha_used"], labels, mind, sse, st["n_corrected"],
                     min_coverage=0.95)


@pytest.mark.parametrize("low,fmt", [(km.KM_LOW_FP16, 0), (km.KM_LOW_BF16, 1)])
def test_small_uniform_low_precision(ctx, low, fmt):
    # no reliability test: every pair by the expanded formula
    n, d, k = 4000, 6, 24
    X, _, _ = W.blobs(n, d, k, seed=90, std=0.5)
    C = W.init_centroids(X, k, 91)
    labels, mind, sse, st = _assign(ctx, dev(X), dev(C), prec(low, km.KM_ALPHA_NONE))
    assert st["n_corrected"] == 0
    check_assignment(X, C, fmt, -1.0, labels, mind, sse, 0, min_coverage=0.9)


def test_small_dense_flags(ctx):
    # every coordinate near 1000: FP16 rounds all of them to the same values,
    # every pair fails the test and is recomputed in FP64
    X, C = W.cancellation_pair(3000, 64, 16, seed=92)
    labels, mind, sse, st = _assign(ctx, dev(X), dev(C), prec())
    assert st["n_corrected"] == 3000 * 64
    check_assignment(X, C, 0, st["alpha_used"], labels, mind, sse, st["n_corrected"],
                     min_coverage=0.99)


def test_small_segmentation_instance(ctx):
    # a segmentation-shaped instance (d = 5, features in [0, 1]) where a
    # tenth of the pairs is flagged
    X, _ = W.segmentation_instance(93, H=160, W=200)
    C = W.init_centroids(X, 48, 94)
    labels, mind, sse, st = _assign(ctx, dev(X), dev(C), prec())
    rep = check_assignment(X, C, 0, st["alpha_used"], labels, mind, sse, st["n_corrected"],
                           min_coverage=0.95)
    assert st["n_corrected"] > 0.01 * X.shape[0] * C.shape[0]
    assert rep["coverage"] > 0.95


def test_small_repeatable_and_outputs_optional(ctx):
    # bitwise-repeatable; labels alone equal the labels of a full call
    n, d, k = 50_000, 5, 64
    X, _, _ = W.blobs(n, d, k, seed=94, std=0.4)
    C = W.init_centroids(X, k, 95)
    Xd, Cd = dev(X), dev(C)
    a = _assign(ctx, Xd, Cd, prec())
    b = _assign(ctx, Xd, Cd, prec())
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    lab, _, _, _ = km.kmeans_assign(ctx, Xd, Cd, prec(), stats=False)
    assert np.array_equal(host(lab), a[0])


def test_small_centre_errors(ctx):
    # the small-problem kernel checks the centres itself (no preparation
    # launch): a non-finite centre and an FP16-overflowing one are reported
    X = np.ones((300, 5), dtype=np.float32)
    C = np.ones((4, 5), dtype=np.float32)
    Cn = C.copy()
    Cn[2, 3] = np.inf
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign(ctx, dev(X), dev(Cn), prec())
    assert e.value.code == -3
    Cr = C.copy()
    Cr[1, 0] = -7.0e4
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign(ctx, dev(X), dev(Cr), prec())
    assert e.value.code == -2
    km.kmeans_assign(ctx, dev(X), dev(Cr), prec(km.KM_LOW_BF16))
