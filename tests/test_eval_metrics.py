"""The clustering agreement measures of the library (host code, no device
work): ARI and AMI against scikit-learn's definitions, and the segmentation
Diff (best one-to-one matching of ids) against a brute force over all
matchings and against SciPy's assignment solver."""

import itertools

import numpy as np
import pytest

km = pytest.importorskip("paper_2407_12208_amd")
sk = pytest.importorskip("sklearn.metrics")
opt = pytest.importorskip("scipy.optimize")


def _pairs(seed):
    g = np.random.default_rng(seed)
    out = []
    for n, ka, kb, flip in ((50, 3, 4, 0.3), (1000, 8, 8, 0.1), (5000, 16, 12, 0.5), (300, 1, 5, 0.0),
                            (20, 20, 20, 0.2), (4000, 64, 64, 0.05)):
        a = g.integers(0, ka, size=n)
        b = a % kb
        m = g.random(n) < flip
        b[m] = g.integers(0, kb, size=int(m.sum()))
        out.append((a.astype(np.int32) * 7 - 3, b.astype(np.int32)))  # arbitrary label values
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_ari_and_ami_match_sklearn(seed):
    for a, b in _pairs(seed):
        assert km.kmeans_ari(a, b) == pytest.approx(sk.adjusted_rand_score(a, b), abs=1e-12)
        assert km.kmeans_ami(a, b) == pytest.approx(sk.adjusted_mutual_info_score(a, b), abs=1e-9)


def test_special_cases():
    one = np.zeros(10, np.int32)
    own = np.arange(10, dtype=np.int32)
    assert km.kmeans_ari(one, one) == 1.0 and km.kmeans_ami(one, one) == 1.0
    assert km.kmeans_ari(own, own) == 1.0 and km.kmeans_ami(own, own) == 1.0
    perm = np.array([2, 2, 0, 0, 1, 1], np.int32)
    ref = np.array([0, 0, 1, 1, 2, 2], np.int32)
    assert km.kmeans_ari(perm, ref) == pytest.approx(1.0)
    assert km.kmeans_ami(perm, ref) == pytest.approx(1.0)
    assert km.kmeans_label_diff(perm, ref) == 0.0


def test_label_diff_brute_force_and_scipy():
    g = np.random.default_rng(5)
    for n, k in ((12, 3), (40, 4), (200, 5)):
        a = g.integers(0, k, size=n).astype(np.int32)
        b = g.integers(0, k, size=n).astype(np.int32)
        best = max(sum(int(np.sum((a == i) & (b == p[i]))) for i in range(k))
                   for p in itertools.permutations(range(k)))
        assert km.kmeans_label_diff(a, b) == pytest.approx(1 - best / n)
    for n, ka, kb in ((3000, 32, 32), (5000, 20, 27)):
        a = g.integers(0, ka, size=n).astype(np.int32)
        b = np.where(g.random(n) < 0.7, a % kb, g.integers(0, kb, size=n)).astype(np.int32)
        cont = np.zeros((ka, kb))
        np.add.at(cont, (a, b), 1)
        r, c = opt.linear_sum_assignment(-cont)
        assert km.kmeans_label_diff(a, b) == pytest.approx(1 - cont[r, c].sum() / n)


def test_bad_arguments():
    with pytest.raises(ValueError):
        km.kmeans_ari(np.zeros(3, np.int32), np.zeros(4, np.int32))
    with pytest.raises(km.KMeansError):
        km.kmeans_ari(np.zeros(0, np.int32), np.zeros(0, np.int32))
