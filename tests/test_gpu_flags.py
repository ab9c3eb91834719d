"""Per-pair fallback decisions of the production assignment kernels (the
large-problem kernel and the small-problem kernel, as kmeans_assign runs them)
against the oracle's per-pair classification (Theorem thm:dist-exp with FP32
arithmetic), through kmeans_assign_flags: no surely kept pair is flagged,
every surely flagged pair is, the ones count equals the corrected-pair
counter, and the labels are kmeans_assign's."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import fp32_classes

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


FP16 = km.Precision(km.KM_LOW_FP16, km.KM_ALPHA_PAPER_EQ, 5.0)
FP16_ALG = km.Precision(km.KM_LOW_FP16, km.KM_ALPHA_PAPER_ALG, 5.0)
BF16 = km.Precision(km.KM_LOW_BF16, km.KM_ALPHA_PAPER_EQ, 5.0)
BF16_HW = km.Precision(km.KM_LOW_BF16, km.KM_ALPHA_HW, 5.0)
FP32 = km.Precision(km.KM_LOW_FP32, km.KM_ALPHA_PAPER_EQ, 5.0)
FMT = {km.KM_LOW_FP16: 0, km.KM_LOW_BF16: 1, km.KM_LOW_FP32: 2}


def check_flags(ctx, X, C, p, hint=None):
    Xd, Cd = dev(X), dev(C)
    lab_ref, _, _, st_ref = km.kmeans_assign(ctx, Xd, Cd, p, stats=True)
    if hint is not None:
        lab, fl, st = km.kmeans_assign_flags(ctx, Xd, Cd, p, labels=dev(hint), labels_hint=True)
    else:
        lab, fl, st = km.kmeans_assign_flags(ctx, Xd, Cd, p)
    lab, fl = host(lab), host(fl).astype(bool)
    np.testing.assert_array_equal(lab, host(lab_ref))
    assert int(fl.sum()) == st["n_corrected"] == st_ref["n_corrected"]
    if FMT[p.low] == 2:  # FP32 operands: O4's rounding is the identity
        cls, _ = fp32_classes(X, C, st["alpha_used"], oracle.dist_rows(X, C))
    else:
        cls = oracle.mp_rows(X, C, FMT[p.low], st["alpha_used"])["cls"]
    # the classification decides nearly every pair (no overflowing inputs here)
    assert np.isin(cls, (-1, 1)).mean() > 0.99, np.unique(cls, return_counts=True)
    assert not np.any(fl & (cls == 1)), "a surely kept pair was flagged"
    assert not np.any(~fl & (cls == -1)), "a surely flagged pair was kept"
    return dict(flagged=int(fl.sum()), sure=int((cls == -1).sum()), amb=int((cls == 0).sum()),
                kept=int((cls == 1).sum()), pairs=fl.size)


@pytest.mark.parametrize("n,d,k,p,data", [
    # large-problem kernel (d > 32 or k > 64)
    (1_500, 128, 300, FP16, "normal"),
    (1_500, 128, 300, FP16, "cancellation"),   # every pair flagged: queue overflow path
    (2_000, 64, 1024, FP16, "blobs"),          # own-blob pairs flagged
    (2_000, 64, 1024, BF16_HW, "blobs"),
    (999, 100, 97, FP16_ALG, "blobs"),         # d off the padded extent, ragged k
    (700, 48, 130, FP32, "blobs"),
    # small-problem kernel (d <= 32, k <= 64)
    (5_000, 5, 40, FP16, "segmentation"),      # a tenth of the pairs flagged
    (20_000, 32, 16, FP16, "blobs"),
    (3_001, 8, 64, BF16, "blobs"),
    (777, 3, 9, FP16, "cancellation"),
])
def test_flags_match_oracle_classification(ctx, n, d, k, p, data):
    if data == "normal":
        X, C = W.gaussian_pair(n, k, d, seed=n + k)
    elif data == "cancellation":
        X, C = W.cancellation_pair(n, k, d, seed=n + k)
    elif data == "segmentation":
        X = W.segmentation_instance(3, H=50, W=100)[0][:n]
        C = W.init_centroids(X, k, 4)
    else:
        X, _, _ = W.blobs(n, d, min(k, 64), seed=n + d, std_range=(0.1, 2.0), center_box=(-50, 50))
        C = W.init_centroids(X, k, 5)
    print("case", n, d, k, p.low, p.alpha_mode, data, flush=True)
    rep = check_flags(ctx, X, C, p)
    print(rep)
    if data == "cancellation":
        assert rep["flagged"] == rep["pairs"]


def test_flags_with_labels_hint(ctx):
    # the large kernel corrects a surely flagged hinted pair before its sweep
    # (and keeps it out of the block test): the decision is recorded there
    X, _, _ = W.blobs(3_000, 64, 128, seed=8, std=0.2)
    C = W.init_centroids(X, 128, 9)
    lab, _, _, _ = km.kmeans_assign(ctx, dev(X), dev(C), FP16, stats=False)
    rep = check_flags(ctx, X, C, FP16, hint=host(lab))
    assert rep["flagged"] > 0


def test_flags_of_routes_without_a_test(ctx):
    X, C = W.gaussian_pair(500, 70, 64, seed=3)
    # no test: nothing flagged
    for p in (km.Precision(km.KM_LOW_FP16, km.KM_ALPHA_NONE), km.Precision(km.KM_EXACT64)):
        _, fl, st = km.kmeans_assign_flags(ctx, dev(X), dev(C), p)
        assert not host(fl).any() and st["n_corrected"] == 0
    # BF16 at the paper's threshold for d = 64 flags every pair (direct kernel)
    p = km.Precision(km.KM_LOW_BF16, km.KM_ALPHA_PAPER_EQ, 5.0)
    assert km.kmeans_alpha(p, 64) >= 2.5
    _, fl, st = km.kmeans_assign_flags(ctx, dev(X), dev(C), p)
    assert host(fl).all() and st["n_corrected"] == 500 * 70
