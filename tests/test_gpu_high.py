"""GPU parity of the other correction precisions (km_precision.high):
FP16/BF16 -> FP32 and the uniform FP16 -> FP16, BF16 -> BF16, FP32 -> FP32
fallbacks (eq:fallback-rule, eq:fallback-rule-mp, the variants of Section
6.1), against O4 for the test and O5 for the corrected values, through the
C ABI.  Corrected values are compared bit for bit: both sides round every
operation once, in the same order."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import check_assignment_high, corr_intervals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
km = pytest.importorskip("paper_2407_12208_amd")

VARIANTS = [(km.KM_LOW_FP16, km.KM_HIGH_FP32), (km.KM_LOW_BF16, km.KM_HIGH_FP32),
            (km.KM_LOW_FP16, km.KM_HIGH_LOW), (km.KM_LOW_BF16, km.KM_HIGH_LOW),
            (km.KM_LOW_FP32, km.KM_HIGH_LOW)]
IDS = ["fp16_fp32", "bf16_fp32", "fp16_fp16", "bf16_bf16", "fp32_fp32"]


@pytest.fixture(scope="module")
def ctx():
    c = km.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def data(kind, n, k, d, seed):
    """normal: N(0, 9) points with a third of the centres placed next to
    points (near pairs, flagged); near: every coordinate 1e3 + 1e-2 z
    (cancellation: every pair is near)."""
    if kind == "near":
        return W.cancellation_pair(n, k, d, seed)
    g = np.random.default_rng(seed)
    X = (g.standard_normal((n, d)) * 3).astype(np.float32)
    C = (g.standard_normal((k, d)) * 3).astype(np.float32)
    idx = g.choice(n, size=k // 3, replace=False)
    C[: k // 3] = X[idx] + (g.standard_normal((k // 3, d)) * 1e-3).astype(np.float32)
    return X, C


@pytest.mark.parametrize("low,high", VARIANTS, ids=IDS)
@pytest.mark.parametrize("kind,n,d,k", [("normal", 1500, 128, 300), ("normal", 2500, 5, 40),
                                        ("near", 1000, 32, 64)])
def test_pairwise_values(ctx, low, high, kind, n, d, k):
    X, C = data(kind, n, k, d, 11 + d)
    pr = km.Precision(low, high=high)
    alpha = km.kmeans_alpha(pr, d)
    D, fl = km.kmeans_pairwise(ctx, dev(X), dev(C), pr, flagged=True)
    D, fl = host(D).astype(np.float64), host(fl).astype(bool)
    fmt = {km.KM_LOW_FP16: 0, km.KM_LOW_BF16: 1, km.KM_LOW_FP32: 2}[low]
    lo, hi, cls, h32, dist = corr_intervals(X, C, fmt, alpha, high)
    assert not np.any(fl & (cls == 1)), "a surely kept pair was corrected"
    assert not np.any(~fl & (cls == -1)), "a surely corrected pair was kept"
    # corrected pairs: O5's value, bit for bit (inf included)
    bad = np.nonzero(fl & (D != h32))
    assert bad[0].size == 0, "corrected value differs at %s: gpu %r, oracle %r" % (
        list(zip(*bad))[:3], D[bad][:3], h32[bad][:3])
    # kept pairs: within the bound of the expanded formula
    kept = ~fl
    assert np.all((D[kept] >= lo[kept]) & (D[kept] <= hi[kept])), "kept pair outside its bound"
    assert fl.any() or kind == "normal"


@pytest.mark.parametrize("low,high", VARIANTS, ids=IDS)
@pytest.mark.parametrize("kind,n,d,k", [("normal", 4000, 128, 256), ("normal", 40000, 5, 40),
                                        ("normal", 20000, 32, 64), ("near", 8000, 5, 16)])
def test_assignment(ctx, low, high, kind, n, d, k):
    X, C = data(kind, n, k, d, 23 + d)
    pr = km.Precision(low, high=high)
    alpha = km.kmeans_alpha(pr, d)
    labels, mindist, _, st = km.kmeans_assign(ctx, dev(X), dev(C), pr, mindist=True, sync=True)
    fmt = {km.KM_LOW_FP16: 0, km.KM_LOW_BF16: 1, km.KM_LOW_FP32: 2}[low]
    rep = check_assignment_high(X, C, fmt, alpha, high, host(labels), host(mindist),
                                st["n_corrected"], min_coverage=0.5 if kind == "normal" else 0.0)
    assert st["n_pairs"] == n * k


@pytest.mark.parametrize("high", [km.KM_HIGH_FP32, km.KM_HIGH_LOW])
def test_batch_equals_alone(ctx, high):
    pr = km.Precision(km.KM_LOW_FP16, high=high)
    insts = [W.blobs(n, d, k, seed) for n, d, k, seed in
             ((6000, 5, 12, 1), (9000, 16, 30, 2), (3000, 128, 20, 3))]
    items, alone = [], []
    for X, _, _ in insts:
        k = {5: 12, 16: 30, 128: 20}[X.shape[1]]
        C0 = W.init_centroids(X, k, 9)
        items.append(km.BatchItem(X=dev(X), C=dev(C0), max_iter=6))
        C1 = dev(C0)
        lab = torch.empty(X.shape[0], dtype=torch.int32, device="cuda")
        km.kmeans_lloyd(ctx, dev(X), C1, 6, prec=pr, labels=lab, stats=False)
        alone.append((C1, lab))
    km.kmeans_solve_batch(ctx, items, pr)
    for it, (C1, lab) in zip(items, alone):
        assert torch.equal(it.labels, lab)
        assert torch.equal(it.C, C1)


def test_exact64_rejects_other_high(ctx):
    X = np.zeros((10, 4), np.float32)
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign(ctx, dev(X), dev(X[:3]), km.Precision(km.KM_EXACT64, high=km.KM_HIGH_FP32), sync=True)
    assert e.value.code == -1


@pytest.mark.parametrize("low,high", VARIANTS, ids=IDS)
def test_every_pair_corrected_runs_the_direct_formula_in_that_precision(ctx, low, high):
    # a threshold that flags every pair (alpha >= 2.5) routes the pass to the
    # direct-formula kernel, in the correction precision
    n, d, k = 3000, 40, 70
    X, C = data("normal", n, k, d, 5)
    pr = km.Precision(low, km.KM_ALPHA_EXPLICIT, alpha=3.0, high=high)
    fmt = {km.KM_LOW_FP16: 0, km.KM_LOW_BF16: 1, km.KM_LOW_FP32: 2}[low]
    h32 = oracle.corr_rows(X, C, high, fmt).astype(np.float32)
    D, fl = km.kmeans_pairwise(ctx, dev(X), dev(C), pr, flagged=True)
    assert bool(host(fl).all())
    np.testing.assert_array_equal(host(D), h32)
    labels, mindist, _, st = km.kmeans_assign(ctx, dev(X), dev(C), pr, mindist=True, sync=True)
    check_assignment_high(X, C, fmt, 3.0, high, host(labels), host(mindist), st["n_corrected"])
    assert st["n_corrected"] == n * k
