"""GPU parity of the assignment pass (kmeans_assign / kmeans_pairwise /
kmeans_quantize) against the CPU oracle, through the C ABI."""

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import check_assignment, check_pairwise

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


def prec(low=km.KM_LOW_FP16, mode=km.KM_ALPHA_PAPER_EQ, rho=5.0, alpha=0.0):
    return km.Precision(low, mode, rho, alpha)


# ---------------------------------------------------------------------------
# Quantisation: bit-exact against the oracle's IEEE round-to-nearest-even
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("low", [km.KM_LOW_FP16, km.KM_LOW_BF16])
def test_quantize_matches_oracle_rne(ctx, low):
    g = np.random.default_rng(7)
    bits = g.integers(0, 2 ** 32, size=1 << 18, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    edge = np.array([0.0, -0.0, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 65519.99,
                     65520.0, 2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -24, 1e-40,
                     3.3895e38, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8], dtype=np.float32)
    x = np.concatenate([x[~np.isnan(x)], edge])
    out = host(km.kmeans_quantize(ctx, dev(x), low)).view(np.uint16)
    ref = oracle.round_low(x, low)
    if low == km.KM_LOW_FP16:
        with np.errstate(over="ignore"):
            ref_bits = ref.astype(np.float16).view(np.uint16)
    else:
        ref_bits = (ref.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    mism = np.nonzero(out != ref_bits)[0]
    assert mism.size == 0, "RNE mismatch for %r" % x[mism[:5]]


def test_alpha_matches_oracle():
    for low, fmt in ((km.KM_LOW_FP16, 0), (km.KM_LOW_BF16, 1)):
        for d in (3, 5, 16, 32, 64, 128):
            for mode, form in ((km.KM_ALPHA_PAPER_EQ, "eq"), (km.KM_ALPHA_PAPER_ALG, "alg")):
                a = km.kmeans_alpha(prec(low, mode), d)
                ref = oracle.alpha_value(fmt, d, 5.0, form)
                if ref < 2.5:
                    assert a == float(np.float32(ref))
                else:
                    assert a == pytest.approx(ref, rel=1e-15)
    assert km.kmeans_alpha(prec(mode=km.KM_ALPHA_NONE), 8) == -1.0


# ---------------------------------------------------------------------------
# Materialised pairs: every value, every flag
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d", [3, 5, 16, 32, 64, 100, 128, 200])
@pytest.mark.parametrize("low,fmt", [(km.KM_LOW_FP16, 0), (km.KM_LOW_BF16, 1)])
def test_pairwise_values_and_flags(ctx, d, low, fmt):
    n, k = 613, 97  # ragged: several tiles plus a tail, a padded centre block
    X, _, _ = W.blobs(n, d, 7, seed=100 + d, std=0.5)
    C = W.init_centroids(X, k, 200 + d)
    p = prec(low)
    alpha = km.kmeans_alpha(p, d)
    D, fl = km.kmeans_pairwise(ctx, dev(X), dev(C), p, flagged=True)
    if alpha >= 2.5:  # dense-fallback route: everything corrected
        assert host(fl).all()
        ref = oracle.dist_rows(X, C)
        np.testing.assert_allclose(host(D), ref, rtol=2 * 2.0 ** -24, atol=0)
        return
    rep = check_pairwise(X, C, fmt, alpha, host(D), host(fl))
    assert rep["n_flagged"] >= rep["n_sure"]


def test_pairwise_uniform_no_fallback(ctx):
    X, C = W.gaussian_pair(300, 70, 64, seed=5)
    p = prec(mode=km.KM_ALPHA_NONE)
    D, fl = km.kmeans_pairwise(ctx, dev(X), dev(C), p, flagged=True)
    assert not host(fl).any()
    r = oracle.mp_rows(X, C, 0, -1.0)
    err = np.abs(host(D).astype(np.float64) - r["q"])
    assert np.all(err <= r["A"])


# ---------------------------------------------------------------------------
# Assignment pass: labels, distances, SSE, corrected-pair count
# ---------------------------------------------------------------------------

def _run_assign(ctx, X, C, p):
    labels, mind, sse, st = km.kmeans_assign(ctx, dev(X), dev(C), p, mindist=True,
                                             sse=True, stats=True)
    return host(labels), host(mind), float(host(sse)[0]), st


@pytest.mark.parametrize("low,fmt", [(km.KM_LOW_FP16, 0), (km.KM_LOW_BF16, 1)])
@pytest.mark.parametrize("shape", [(20000, 32, 16), (5000, 5, 37), (3001, 64, 200),
                                   (2000, 128, 300), (777, 3, 8), (1500, 200, 64)])
def test_assign_blobs(ctx, low, fmt, shape):
    n, d, k = shape
    X, _, _ = W.blobs(n, d, k, seed=n + d + k)
    C = W.init_centroids(X, k, 11)
    p = prec(low)
    labels, mind, sse, st = _run_assign(ctx, X, C, p)
    assert st["data_status"] == 0
    assert st["n_pairs"] == n * k
    rep = check_assignment(X, C, fmt, st["alpha_used"], labels, mind, sse,
                           st["n_corrected"], min_coverage=0.95)
    assert rep["coverage"] > 0.95


def test_assign_lloyd_small_workload(ctx):
    # 20,000 points, d = 32, 16 blobs: the single-solve workload's first pass
    cfg = W.LLOYD_SMALL
    X, _, _ = W.blobs(cfg["n"], cfg["d"], cfg["k"], cfg["seed"])
    C = W.init_centroids(X, cfg["k"], cfg["init_seed"])
    labels, mind, sse, st = _run_assign(ctx, X, C, prec())
    rep = check_assignment(X, C, 0, st["alpha_used"], labels, mind, sse,
                           st["n_corrected"], min_coverage=0.99)
    assert st["n_corrected"] > 0  # own-blob pairs fail the test at d = 32


@pytest.mark.parametrize("low,fmt", [(km.KM_LOW_FP16, 0), (km.KM_LOW_BF16, 1)])
def test_assign_cancellation_prone(ctx, low, fmt):
    # every coordinate 1e3 + 1e-2 z: every pair fails the test
    X, C = W.cancellation_pair(2000, 100, 128, seed=77)
    labels, mind, sse, st = _run_assign(ctx, X, C, prec(low))
    check_assignment(X, C, fmt, st["alpha_used"], labels, mind, sse,
                     st["n_corrected"], min_coverage=0.99)
    assert st["n_corrected"] == 2000 * 100


def test_assign_near_duplicates(ctx):
    # Section 6.1.2 construction: only the near pairs are corrected
    P, C, near = W.near_duplicates(1000, 128, seed=9, fraction=0.5)
    p = prec(mode=km.KM_ALPHA_PAPER_ALG)
    labels, mind, sse, st = _run_assign(ctx, P, C, p)
    assert st["n_corrected"] == len(near)
    check_assignment(P, C, 0, st["alpha_used"], labels, mind, sse, st["n_corrected"])
    np.testing.assert_array_equal(labels[near], near)


def test_collinear_cancellation_closed_form(ctx):
    # x_i = 1000 + i e_1: blocks of m points; labels floor(i/m), distances exact
    k, m, d = 8, 10, 16
    X, v, a = W.collinear(k, m, d, offset=1000.0)
    Cfix = np.array([a + ((m - 1) / 2 + j * m) * v for j in range(k)], dtype=np.float32)
    labels, mind, sse, st = _run_assign(ctx, X, Cfix, prec())
    i = np.arange(k * m)
    np.testing.assert_array_equal(labels, i // m)
    np.testing.assert_array_equal(mind, ((i - (m - 1) / 2 - (i // m) * m) ** 2).astype(np.float32))
    assert sse == k * m * (m * m - 1) / 12


def test_exact64_baseline(ctx):
    X, _, _ = W.blobs(3000, 40, 50, seed=3)
    C = W.init_centroids(X, 50, 4)
    labels, mind, sse, st = _run_assign(ctx, X, C, prec(km.KM_EXACT64))
    assert st["n_corrected"] == 0
    check_assignment(X, C, None, None, labels, mind, sse, None, min_coverage=0.999)
    ol, om, osse = oracle.assign(X, C)
    assert (labels == ol).mean() > 0.999


def test_alpha_infinity_is_fp64_direct(ctx):
    # alpha = inf corrects every pair: labels follow the FP64 direct values
    # rounded to FP32 and mindist is the FP64 value rounded once
    X, _, _ = W.blobs(2500, 24, 30, seed=12)
    C = W.init_centroids(X, 30, 13)
    labels, mind, sse, st = _run_assign(ctx, X, C, prec(mode=km.KM_ALPHA_EXPLICIT, alpha=1e30))
    assert st["n_corrected"] == X.shape[0] * C.shape[0]
    D = oracle.dist_rows(X, C)
    D32 = D.astype(np.float32)
    ref = np.argmin(D32, axis=1)
    np.testing.assert_array_equal(labels, ref)
    d_lab = D[np.arange(len(X)), labels]
    assert np.all(np.abs(mind - d_lab) <= 2.0 ** -24 * d_lab * 2)


def test_fp32_uniform_and_fallback(ctx):
    X, _, _ = W.blobs(3000, 64, 40, seed=21)
    C = W.init_centroids(X, 40, 22)
    for mode in (km.KM_ALPHA_NONE, km.KM_ALPHA_PAPER_EQ):
        p = prec(km.KM_LOW_FP32, mode)
        labels, mind, sse, st = _run_assign(ctx, X, C, p)
        check_assignment(X, C, 2, st["alpha_used"], labels, mind, sse,
                         st["n_corrected"], min_coverage=0.99)


def test_tiny_and_degenerate_shapes(ctx):
    g = np.random.default_rng(1)
    for n, d, k in ((1, 1, 1), (5, 2, 9), (31, 7, 1), (33, 17, 3), (64, 1, 64)):
        X = g.standard_normal((n, d)).astype(np.float32)
        C = g.standard_normal((k, d)).astype(np.float32)
        labels, mind, sse, st = _run_assign(ctx, X, C, prec())
        check_assignment(X, C, 0, st["alpha_used"], labels, mind, sse, st["n_corrected"])


def test_duplicate_centres_pick_lowest_index(ctx):
    X, _, _ = W.blobs(4000, 16, 8, seed=31)
    C = W.init_centroids(X, 8, 32)
    C = np.concatenate([C, C])  # centres 8..15 duplicate 0..7
    labels, mind, sse, st = _run_assign(ctx, X, C, prec())
    assert labels.max() < 8


def test_zero_points_and_centres(ctx):
    X = np.zeros((100, 8), dtype=np.float32)
    C = np.zeros((3, 8), dtype=np.float32)
    labels, mind, sse, st = _run_assign(ctx, X, C, prec())
    assert np.all(labels == 0) and np.all(mind == 0) and sse == 0.0
    assert st["n_corrected"] == 300  # d^ = 0 <= alpha * 0: corrected (strict test)


def test_nonfinite_and_range_errors(ctx):
    X = np.ones((50, 4), dtype=np.float32)
    C = np.ones((2, 4), dtype=np.float32)
    Xn = X.copy()
    Xn[7, 2] = np.nan
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign(ctx, dev(Xn), dev(C), prec())
    assert e.value.code == -3
    Xr = X.copy()
    Xr[3, 1] = 7.0e4
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign(ctx, dev(Xr), dev(C), prec())
    assert e.value.code == -2
    # BF16 has FP32's exponent range: no range error
    km.kmeans_assign(ctx, dev(Xr), dev(C), prec(km.KM_LOW_BF16))


def test_argument_errors(ctx):
    X = dev(np.ones((10, 4), dtype=np.float32))
    C = dev(np.ones((2, 4), dtype=np.float32))
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign(ctx, X, C, prec(rho=1.5))
    assert e.value.code == -1
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign(ctx, X, C, prec(low=9))
    assert e.value.code == -1
    big = dev(np.ones((4, 300), dtype=np.float32))
    with pytest.raises(km.KMeansError) as e:
        km.kmeans_assign(ctx, big, dev(np.ones((2, 300), dtype=np.float32)), prec())
    assert e.value.code == -8


# ---------------------------------------------------------------------------
# Seeding from an earlier assignment (KM_LABELS_HINT) changes nothing
# ---------------------------------------------------------------------------

def _hint_cases():
    g = np.random.default_rng(31)
    X, _, _ = W.blobs(30000, 128, 300, seed=31)
    C = W.init_centroids(X, 300, 32)
    yield "blobs128", X, C, km.KM_LOW_FP16
    Xg, Cg = W.gaussian_pair(20000, 1000, 64, seed=33)
    yield "gauss64_bf16", Xg, Cg, km.KM_LOW_BF16
    yield "gauss64_fp32", Xg[:5000], Cg[:300], km.KM_LOW_FP32
    Xc, Cc = W.cancellation_pair(8000, 64, 16, seed=34)
    yield "cancel16", Xc, Cc, km.KM_LOW_FP16
    # duplicated centres (exact ties) in different 32-centre blocks
    Cd = C.copy()
    Cd[100:140] = Cd[0:40]
    yield "duplicates", X[:8000], Cd, km.KM_LOW_FP16
    # every point close to its own centre compared with the norms: the pair
    # of the (previous) label is the one flagged pair of nearly every point,
    # and a correct hint has it corrected before the sweep
    Xl, _, _ = W.blobs(20000, 64, 256, seed=35, center_box=(-50, 50), std_range=(0.1, 2.0))
    Cl = W.init_centroids(Xl, 256, 36)
    yield "near_own_centre_fp16", Xl, Cl, km.KM_LOW_FP16
    yield "near_own_centre_bf16_hw", Xl, Cl, (km.KM_LOW_BF16, km.KM_ALPHA_HW)
    Xs, _, _ = W.blobs(12000, 40, 100, seed=37, center_box=(-50, 50), std_range=(0.1, 2.0))
    yield "near_own_centre_d40", Xs, W.init_centroids(Xs, 100, 38), km.KM_LOW_FP16


@pytest.mark.parametrize("case", list(range(8)))
def test_labels_hint_gives_identical_results(ctx, case):
    name, X, C, low = list(_hint_cases())[case]
    p = prec(*low) if isinstance(low, tuple) else prec(low)
    Xd, Cd = dev(X), dev(C)
    lab0, md0, sse0, st0 = km.kmeans_assign(ctx, Xd, Cd, p, mindist=True, sse=True)
    n, k = X.shape[0], C.shape[0]
    g = np.random.default_rng(case)
    hints = {
        "same": host(lab0),
        "random": g.integers(0, k, size=n).astype(np.int32),
        "out_of_range": np.where(g.random(n) < 0.5, -3, k + 5).astype(np.int32),
        "shifted": ((host(lab0) + 1) % k).astype(np.int32),
    }
    for hname, h in hints.items():
        lab = dev(h)
        _, md, sse, st = km.kmeans_assign(ctx, Xd, Cd, p, labels=lab, mindist=True, sse=True,
                                          labels_hint=True)
        np.testing.assert_array_equal(host(lab), host(lab0), err_msg="%s/%s" % (name, hname))
        np.testing.assert_array_equal(host(md), host(md0))
        assert float(host(sse)[0]) == float(host(sse0)[0])
        assert st["n_corrected"] == st0["n_corrected"]


# ---------------------------------------------------------------------------
# Exact ties between centres of different norms, and large k
# ---------------------------------------------------------------------------

def _tie_case(i_a, i_b, k, d=128):
    """Points x = e1 and two centres 12 e1 (index i_a, norm 144) and -10 e1
    (index i_b, norm 100) with the same W = x.c - |c|^2/2 = -60 exactly (both
    pairs are kept by the test, d^ = 121); the other centres are far away.
    The lower index must win wherever the two sit (same or different
    32-centre blocks, either order)."""
    n = 1000
    X = np.zeros((n, d), dtype=np.float32)
    X[:, 0] = 1.0
    C = np.zeros((k, d), dtype=np.float32)
    for j in range(k):
        C[j, 1 + j % (d - 1)] = 100.0
    C[i_a] = 0.0
    C[i_a, 0] = 12.0
    C[i_b] = 0.0
    C[i_b, 0] = -10.0
    return X, C


@pytest.mark.parametrize("low", [km.KM_LOW_FP16, km.KM_LOW_BF16])
@pytest.mark.parametrize("i_a,i_b,k", [(3, 150, 200), (150, 3, 200), (0, 1, 2), (1, 0, 2),
                                       (4099, 5, 4100), (33, 32, 64)])
def test_equal_maxima_of_different_norms_pick_lowest_index(ctx, low, i_a, i_b, k):
    X, C = _tie_case(i_a, i_b, k)
    p = prec(low)
    labels, mind, sse, st = _run_assign(ctx, X, C, p)
    assert st["data_status"] == 0
    assert np.all(labels == min(i_a, i_b))
    assert np.all(mind == 121.0)
    n = X.shape[0]
    # seeded with the tied centre of the larger index, or with random labels
    for h in (np.full(n, max(i_a, i_b), dtype=np.int32),
              np.random.default_rng(k).integers(0, k, size=n).astype(np.int32)):
        lab = dev(h)
        km.kmeans_assign(ctx, dev(X), dev(C), p, labels=lab, labels_hint=True)
        assert np.all(host(lab) == min(i_a, i_b))


@pytest.mark.parametrize("k,d", [(4100, 16), (9000, 8), (4096, 32)])
def test_assign_many_centres(ctx, k, d):
    # k of several thousand centres with a ragged last 64-centre tile (4100)
    Xg, Cg = W.gaussian_pair(1500, k, d, seed=k + d)
    for low, fmt in ((km.KM_LOW_FP16, 0), (km.KM_LOW_BF16, 1)):
        labels, mind, sse, st = _run_assign(ctx, Xg, Cg, prec(low))
        assert st["data_status"] == 0
        check_assignment(Xg, Cg, fmt, st["alpha_used"], labels, mind, sse, st["n_corrected"],
                         min_coverage=0.95)
