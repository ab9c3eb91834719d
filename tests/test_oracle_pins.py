"""Pins of the CPU oracle against facts the paper and mathematics fix.

Every check here is independent of the oracle's own code: printed table
values (tests/golden), library conversions (numpy float16, torch bfloat16),
exact rational arithmetic, closed forms and invariants.  Each pin is chosen so
that a plausible slip in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a wrong rounding rule) fails at least one of them.
"""

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------------------
# Table 1: format parameters
# ---------------------------------------------------------------------------

def _sig3(x):
    return float("%.2e" % x)


@pytest.mark.parametrize("row", _golden("table1_formats.txt"))
def test_format_table(row):
    name, u, xmin, xmax, t, emin, emax = row
    fmt = {"fp16": 0, "bf16": 1, "fp32": 2, "fp64": 3}[name]
    assert oracle.fmt_params(fmt) == (int(t), int(emin), int(emax))
    assert _sig3(oracle.unit_roundoff(fmt)) == float(u)
    assert _sig3(oracle.fmt_min_normal(fmt)) == float(xmin)
    assert _sig3(oracle.fmt_max(fmt)) == float(xmax)


def test_gamma_closed_form():
    # gamma_m = m u / (1 - m u) as an exact rational for dyadic u
    for m in (1, 3, 130):
        for t in (8, 11, 24):
            u = Fraction(1, 2 ** t)
            want = m * u / (1 - m * u)
            assert oracle.gamma(m, float(u)) == pytest.approx(float(want), rel=1e-15)
    assert oracle.gamma(2, 0.5) == float("inf")
    assert oracle.gamma(256, 2.0 ** -8) == float("inf")


# ---------------------------------------------------------------------------
# Round to nearest even into FP16 / BF16 against library conversions
# ---------------------------------------------------------------------------

def _bit_sample(count, seed):
    g = np.random.default_rng(seed)
    bits = g.integers(0, 2 ** 32, size=count, dtype=np.uint64).astype(np.uint32)
    return bits.view(np.float32)


def _edge_values():
    v = [0.0, -0.0, 1.0, -1.0, 65504.0, 65505.0, 65519.0, 65519.996, 65520.0,
         65536.0, 1e5, -1e5, 2.0 ** -14, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26,
         2.0 ** -26, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 1 + 2.0 ** -8,
         1 + 3 * 2.0 ** -8, 3.3895e38, 3.4e38, np.inf, -np.inf, 1e-40, -1e-45]
    return np.array(v, dtype=np.float32)


def test_rne_fp16_matches_numpy():
    x = np.concatenate([_bit_sample(1 << 18, 11), _edge_values()])
    x = x[~np.isnan(x)]
    got = oracle.round_low(x, 0)
    with np.errstate(over="ignore"):
        want = x.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(got, want)
    # the sign of zero is kept
    assert np.array_equal(np.signbit(got), np.signbit(want))


def test_rne_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.concatenate([_bit_sample(1 << 18, 12), _edge_values()])
    x = x[~np.isnan(x)]
    got = oracle.round_low(x, 1)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, want)


def test_rne_ties_and_overflow_by_definition():
    f16 = lambda v: float(oracle.round_low(np.float32(v), 0))
    assert f16(1 + 2.0 ** -11) == 1.0                     # tie -> even
    assert f16(1 + 3 * 2.0 ** -11) == 1 + 2.0 ** -9       # tie -> even (up)
    assert f16(65519.99) == 65504.0
    assert f16(65520.0) == float("inf")                   # halfway to 2^16
    assert f16(2.0 ** -25) == 0.0                         # tie with zero
    assert f16(3 * 2.0 ** -26) == 2.0 ** -24              # subnormal quantum
    assert oracle.round_low(np.float32(np.nan), 0) != oracle.round_low(np.float32(np.nan), 0)


# ---------------------------------------------------------------------------
# O1: distances and argmin against exact rationals
# ---------------------------------------------------------------------------

def test_sqdist_within_theorem_bound():
    # Theorem thm:dist-diff: |fl(d^2) - d^2| <= gamma_{r+2} d^2, here in FP64;
    # cancellation-prone inputs (large offset, tiny spread) included.
    g = np.random.default_rng(3)
    u64 = oracle.unit_roundoff(3)
    for trial in range(60):
        d = int(g.integers(1, 24))
        off = [0.0, 1.0, 1e3, 1e6][trial % 4]
        x = (off + g.standard_normal(d) * 10.0 ** -g.integers(0, 5)).astype(np.float32)
        y = (off + g.standard_normal(d) * 10.0 ** -g.integers(0, 5)).astype(np.float32)
        exact = brute.sqdist(x, y)
        got = Fraction(oracle.sqdist(x, y))
        bound = Fraction(oracle.gamma(d + 2, u64)) * exact
        assert abs(got - exact) <= bound


def test_assign_matches_exhaustive_argmin_with_ties():
    g = np.random.default_rng(5)
    for trial in range(20):
        n, k, d = 14, 6, 3
        # coarse dyadic grid: FP64 distances are exact, ties are real
        X = (g.integers(-4, 5, size=(n, d)) / 2.0).astype(np.float32)
        C = (g.integers(-4, 5, size=(k, d)) / 2.0).astype(np.float32)
        C[3] = C[1]  # duplicated centre: an exact tie
        labels, mind, sse = oracle.assign(X, C)
        D = brute.dist_matrix(X, C)
        for i in range(n):
            j = brute.argmin_lowest(D[i])
            assert labels[i] == j
            assert Fraction(mind[i]) == D[i][j]
        assert Fraction(sse) == sum((D[i][labels[i]] for i in range(n)), Fraction(0))
        # the duplicate centre with the larger index is never chosen
        assert not np.any(labels == 3)


def test_dist_rows_orientation():
    # D[i, j] is point i against centre j (a transposed result fails here)
    X = np.array([[0, 0], [3, 4], [1, 1]], dtype=np.float32)
    C = np.array([[0, 0], [1, 0]], dtype=np.float32)
    D = oracle.dist_rows(X, C)
    np.testing.assert_array_equal(D, [[0, 1], [25, 20], [2, 1]])


def test_pairwise_sum_exact_on_integers():
    v = np.arange(1, 10001, dtype=np.float64)
    assert oracle.pairwise_sum(v) == 10000 * 10001 / 2


def test_sse_labels_exact_on_dyadic_data_and_matches_argmin_sse():
    # eq:sse for given labels: with dyadic coordinates every squared
    # difference and every sum is exact in FP64, so the oracle must equal the
    # exact rational sum computed term by term here
    g = np.random.default_rng(21)
    n, d, k = 30, 3, 4
    X = (g.integers(-40, 41, size=(n, d)) / 8.0).astype(np.float32)
    C = (g.integers(-40, 41, size=(k, d)) / 8.0).astype(np.float32)
    labels = g.integers(0, k, size=n).astype(np.int32)
    want = sum(sum((Fraction(float(X[i, l])) - Fraction(float(C[labels[i], l]))) ** 2
                   for l in range(d)) for i in range(n))
    assert oracle.sse_labels(X, C, labels) == float(want)
    # with the nearest-centre labels it is the SSE of O1
    lab, _, sse = oracle.assign(X, C)
    assert oracle.sse_labels(X, C, lab) == sse
    with pytest.raises(ValueError):
        oracle.sse_labels(X, C, np.full(n, k, np.int32))


# ---------------------------------------------------------------------------
# O2: centre update
# ---------------------------------------------------------------------------

def test_update_exact_means_and_empty_cluster():
    g = np.random.default_rng(9)
    n, d, k = 40, 4, 5
    X = (g.integers(-20, 21, size=(n, d)) / 4.0).astype(np.float32)
    labels = g.integers(0, k - 1, size=n).astype(np.int32)  # cluster k-1 empty
    C_old = g.standard_normal((k, d)).astype(np.float32)
    C_new, counts, shift, empty = oracle.update(X, labels, C_old)
    assert empty == 1
    np.testing.assert_array_equal(C_new[k - 1], C_old[k - 1])
    for j in range(k - 1):
        pts = [X[i] for i in range(n) if labels[i] == j]
        assert counts[j] == len(pts)
        mu = brute.mean(pts)
        # exact rational mean, rounded once to FP32
        want = np.array([np.float32(float(v)) for v in mu])
        np.testing.assert_array_equal(C_new[j], want)
    want_shift = max(np.sqrt(((C_new.astype(np.float64) - C_old) ** 2).sum(1)))
    assert shift == pytest.approx(want_shift, rel=1e-15)


def test_update_satisfies_arthur_vassilvitskii_identity():
    # Lemma eq:converge: phi(p,S) = phi(mu,S) + |S| d(p,mu)^2 with mu the mean.
    # With the exact mean the identity is exact; the oracle's centre differs
    # from mu only by the final FP32 rounding, so phi(c_hat) - phi(mu) equals
    # |S| ||c_hat - mu||^2 exactly and is tiny.
    g = np.random.default_rng(10)
    X = (g.standard_normal((25, 3)) * 3 + 1).astype(np.float32)
    labels = np.zeros(25, dtype=np.int32)
    p = g.standard_normal((1, 3)).astype(np.float32)
    C_new, counts, _, _ = oracle.update(X, labels, p)
    mu = brute.mean(list(X))
    phi = lambda c: sum((brute.sqdist_exact_center(x, c) for x in X), Fraction(0))
    pe = [Fraction(float(v)) for v in p[0]]
    assert phi(pe) == phi(mu) + 25 * brute.sqdist_exact_center(p[0], mu)
    ch = [Fraction(float(v)) for v in C_new[0]]
    gap = phi(ch) - phi(mu)
    assert gap == 25 * sum(((a - b) ** 2 for a, b in zip(ch, mu)), Fraction(0))
    u32 = Fraction(oracle.unit_roundoff(2))
    assert gap <= 25 * u32 ** 2 * sum((v * v for v in mu), Fraction(0))


# ---------------------------------------------------------------------------
# O3: Lloyd against exhaustive optimal partitions, fixed points, closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_lloyd_vs_optimal_partition(seed):
    g = np.random.default_rng(seed)
    n, k = 8, 3
    X = (g.integers(-8, 9, size=(n, 2)) / 2.0).astype(np.float32)
    best_sse, best_lab, best_means = brute.optimal_partition(X, k)
    # Lloyd from every k-subset start never beats the optimum
    for start in ([0, 1, 2], [2, 5, 7], [1, 3, 6]):
        res = oracle.lloyd(X, X[start], max_iter=30)
        assert Fraction(res["sse_hist"][-1]) >= best_sse - Fraction(1, 10 ** 9)
    # the optimal partition's means form a Lloyd fixed point
    C0 = np.array([[np.float32(float(v)) for v in mu] for mu in best_means])
    res = oracle.lloyd(X, C0, max_iter=1)
    D = brute.dist_matrix(X, C0)
    want = [brute.argmin_lowest(r) for r in D]
    np.testing.assert_array_equal(res["labels"], want)
    np.testing.assert_allclose(res["C"], C0, rtol=2 ** -23, atol=0)
    assert res["sse_hist"][-1] == pytest.approx(float(best_sse), rel=1e-6)


@pytest.mark.parametrize("offset,direction", [(0.0, "e1"), (1000.0, "e1"),
                                              (0.0, "e12"), (1000.0, "e12")])
def test_collinear_closed_form(offset, direction):
    # x_i = a + i v, i < k*m, m even: contiguous blocks of m are a Lloyd fixed
    # point with centres a + ((m-1)/2 + j m) v and SSE = k m (m^2-1)/12 |v|^2.
    k, m, d = 5, 6, 4
    X, v, a = W.collinear(k, m, d, offset=offset, direction=direction)
    v2 = float(v @ v)
    Cfix = np.array([a + ((m - 1) / 2 + j * m) * v for j in range(k)], dtype=np.float32)
    labels, mind, sse = oracle.assign(X, Cfix)
    i = np.arange(k * m)
    np.testing.assert_array_equal(labels, i // m)
    np.testing.assert_array_equal(mind, (i - (m - 1) / 2 - (i // m) * m) ** 2 * v2)
    assert sse == k * m * (m * m - 1) / 12 * v2
    # a start shifted by +0.25 v returns to the fixed point in one update
    res = oracle.lloyd(X, Cfix + np.float32(0.25) * v.astype(np.float32), max_iter=1)
    np.testing.assert_array_equal(res["C"], Cfix)
    np.testing.assert_array_equal(res["labels"], i // m)


def test_lloyd_sse_never_increases_beyond_rounding_slack():
    # Theorems thm:center-energy-perturb / theorem:center-update-descent: with
    # exact means the SSE never increases; rounding the centres to FP32 can
    # add at most sum_j m_j ||fl32(mu_j) - mu_j||^2 <= n d u32^2 max|mu|^2.
    X, _, _ = W.blobs(3000, 8, 6, seed=21, std=2.5)
    C0 = W.init_centroids(X, 6, 22)
    res = oracle.lloyd(X, C0, max_iter=25)
    h = res["sse_hist"]
    u32 = oracle.unit_roundoff(2)
    slack = X.shape[0] * X.shape[1] * u32 ** 2 * float(np.abs(X).max()) ** 2
    assert np.all(np.diff(h) <= slack + 1e-12 * h[:-1])
    assert h[-1] < h[0]


def test_lloyd_tolerance_stops_early():
    X, _, _ = W.blobs(2000, 4, 3, seed=31)
    C0 = W.init_centroids(X, 3, 32)
    res = oracle.lloyd(X, C0, max_iter=100, tol=1e-8)
    assert res["iters"] < 100
    assert res["shift_hist"][-1] < 1e-8
    assert np.all(res["shift_hist"][:-1] >= 1e-8)
    # tol = 0 never stops early (strict comparison)
    res0 = oracle.lloyd(X, C0, max_iter=7, tol=0.0)
    assert res0["iters"] == 7 and len(res0["sse_hist"]) == 8


# ---------------------------------------------------------------------------
# O4: the mixed-precision reliability test, emulated
# ---------------------------------------------------------------------------

def test_mp_quantised_distance_exact_on_tiny_inputs():
    g = np.random.default_rng(41)
    X = (g.standard_normal((5, 6)) * 3).astype(np.float32)
    C = (g.standard_normal((4, 6)) * 3).astype(np.float32)
    for fmt, lib_round in ((0, lambda a: a.astype(np.float16)),
                           (1, None)):
        r = oracle.mp_rows(X, C, fmt, 0.5)
        if lib_round is None:
            torch = pytest.importorskip("torch")
            lib_round = lambda a: torch.from_numpy(a).to(torch.bfloat16).float().numpy()
        Xq, Cq = lib_round(X), lib_round(C)
        for i in range(5):
            for j in range(4):
                q = brute.sqdist(Xq[i], Cq[j])
                assert abs(Fraction(r["q"][i, j]) - q) <= Fraction(1e-14) * q
                S = brute.sqdist(Xq[i], np.zeros(6)) + brute.sqdist(Cq[j], np.zeros(6))
                assert abs(Fraction(r["S"][i, j]) - S) <= Fraction(1e-14) * S
                assert r["dist"][i, j] == oracle.sqdist(X[i], C[j])


def test_mp_alpha_at_least_two_corrects_everything():
    # d^ <= 2(||x~||^2 + ||c~||^2) always, so alpha >= 2 sends every pair to
    # the direct formula; BF16 at d = 128 under the equation-form threshold
    # is such a case, matching the 100% fallback the paper prints for BF16.
    rows = _golden("bf16_eta_d128.txt")
    d = int(rows[0][0])
    a = oracle.alpha_value(1, d, 5.0, "eq")
    assert a >= 2.0
    X, C = W.gaussian_pair(64, 200, d, seed=43)
    c = oracle.mp_count(X, C, 1, a)
    assert c[2] == 0 and c[0] + c[1] == X.shape[0] * C.shape[0]
    assert float(rows[0][2]) == 100.0 * (c[0] + c[1]) / c.sum()
    # and alpha = 3 on generic data: every pair surely corrected
    c3 = oracle.mp_count(X, C, 0, 3.0)
    assert c3[0] == X.shape[0] * C.shape[0]


def test_mp_near_far_stress_reproduces_printed_eta():
    # Table tab:dist-streess-test, FP16->FP64 with rho = 5: only the
    # near-duplicate pairs fall back.  Under the listing form of the threshold
    # (alpha = rho gamma) our construction at the paper's size reproduces the
    # printed eta for every fraction; under the equation form (twice as large)
    # the near pairs are still all flagged, plus a few far pairs.
    m, d = 5000, 128
    a_alg = oracle.alpha_value(0, d, 5.0, "alg")
    a_eq = oracle.alpha_value(0, d, 5.0, "eq")
    for f_pct, eta_pct in _golden("stress_eta.txt"):
        f = float(f_pct) / 100.0
        if f not in (0.0, 1.0):
            continue  # keep the CPU suite short; 0% and 100% bracket the rest
        P, C, near = W.near_duplicates(m, d, seed=45, fraction=f)
        c = oracle.mp_count(P, C, 0, a_alg)
        assert c[1] == 0
        eta = 100.0 * c[0] / c.sum()
        assert round(eta, 2) == float(eta_pct)
        assert c[0] == len(near)


def test_mp_near_duplicates_flag_exactly_the_near_pairs():
    m, d = 300, 128
    P, C, near = W.near_duplicates(m, d, seed=47, fraction=0.5)
    a = oracle.alpha_value(0, d, 5.0, "alg")
    r = oracle.mp_rows(P, C, 0, a)
    flagged = np.argwhere(r["cls"] == -1)
    assert sorted(map(tuple, flagged)) == [(i, i) for i in near]
    assert not np.any(r["cls"] == 0)


def test_mp_kept_pairs_obey_quantisation_bound():
    # Section 4.3: a pair that passes the test with rho~ > 2 has
    # |q - d^2| <= C(x,y) <= E^l and relative error <= 2/(rho~ - 2).
    X, C = W.gaussian_pair(200, 300, 32, seed=49)
    rho = 5.0
    a = oracle.alpha_value(0, 32, rho, "eq")
    r = oracle.mp_rows(X, C, 0, a)
    kept = r["cls"] == 1
    assert kept.sum() > 0.9 * kept.size
    rel = np.abs(r["q"][kept] - r["dist"][kept]) / r["dist"][kept]
    assert rel.max() <= 2.0 / (rho - 2.0)
    # the a-posteriori bound for kept pairs never exceeds twice E^l
    El = (a / rho) * r["S"][kept]
    assert np.all(r["B"][kept] <= 2 * El)
    # corrected pairs: bound is FP32 rounding of the FP64 direct value
    u32 = oracle.unit_roundoff(2)
    corr = r["cls"] == -1
    np.testing.assert_allclose(r["B"][corr], 2 * u32 * r["dist"][corr])


def test_mp_overflow_is_reported():
    X = np.array([[1.0, 70000.0]], dtype=np.float32)
    C = np.array([[1.0, 2.0], [0.0, 0.0]], dtype=np.float32)
    r = oracle.mp_rows(X, C, 0, 0.5)
    assert r["n_bad"] == 2 and np.all(r["cls"] == -2)
    r = oracle.mp_rows(X, C, 1, 0.5)  # BF16 has FP32's range
    assert r["n_bad"] == 0


def test_label_gate_logic():
    dist = np.array([[1.0, 1.5, 3.0], [2.0, 2.001, 5.0]])
    B = np.full_like(dist, 0.1)
    gated = oracle.label_gate(dist, B, np.array([0, 0]))
    assert gated.tolist() == [True, False]


def _fp32_expanded(X, C, fmt):
    """Expanded formula of the rounded inputs evaluated in float32 (numpy's
    summation order; the products of FP16/BF16 values are exact in FP32)."""
    Xq = oracle.round_low(X, fmt).astype(np.float32)
    Cq = oracle.round_low(C, fmt).astype(np.float32)
    nx = (Xq * Xq).sum(axis=1, dtype=np.float32)
    nc = (Cq * Cq).sum(axis=1, dtype=np.float32)
    G = (Xq @ Cq.T).astype(np.float32)
    dh = np.maximum(nx[:, None] + nc[None, :] - np.float32(2) * G, np.float32(0))
    S = nx[:, None].astype(np.float64) + nc[None, :].astype(np.float64)
    return dh.astype(np.float64), S


def _boundary_pairs(d, seed):
    # points at log-uniform distances 1e-4..10 from centres in [-10, 10]^d:
    # the test's threshold falls inside the range, on both sides
    g = np.random.default_rng(seed)
    C = g.uniform(-10, 10, size=(24, d)).astype(np.float32)
    owner = g.integers(0, 24, size=600)
    delta = 10.0 ** g.uniform(-4, 1, size=(600, 1))
    z = g.standard_normal((600, d))
    X = (C[owner].astype(np.float64) + delta * z / np.sqrt(d)).astype(np.float32)
    return X, C


def _aligned_pairs(d, fmt, seed):
    # coordinates in [8, 16): c rounds down by ~ulp/2, x = c + (j + 0.1) ulp
    # rounds up by ~ulp/2, so the rounded difference is (j + 1) ulp in every
    # coordinate: the quantisation error has the sign of the difference
    g = np.random.default_rng(seed)
    ulp = 16.0 * oracle.unit_roundoff(fmt)  # spacing of the format in [8, 16)
    rows_x, rows_c = [], []
    for j in range(1, 41):
        m = g.integers(0, int(4 / ulp), size=d)
        c = 8.0 + (m + 0.45) * ulp
        x = 8.0 + (m + j + 0.55) * ulp
        rows_x.append(x)
        rows_c.append(c)
    return np.array(rows_x, dtype=np.float32), np.array(rows_c, dtype=np.float32)


@pytest.mark.parametrize("fmt", [oracle.FP16, oracle.BF16])
@pytest.mark.parametrize("d", [5, 64, 128])
def test_hw_alpha_kept_pairs_obey_relative_bound(fmt, d):
    # Section 4.3's decomposition (arithmetic error of the expanded formula
    # plus the conversion error of the rounded inputs) with FP32 accumulation:
    # a pair whose FP32 expanded value passes d^ > alpha_hw * S is within
    # 1/(rho - 1) of the exact distance of the FP32 inputs
    rho = 5.0
    a = oracle.alpha_value(fmt, d, rho, "hw")
    a_bad = rho * 2.0 * oracle.gamma(d + 2, 2.0 ** -23)  # conversion term dropped
    X, C = _boundary_pairs(d, 40 + d + fmt)
    dh, S = _fp32_expanded(X, C, fmt)
    exact = oracle.dist_rows(X, C)
    kept = dh > a * S
    assert 0.05 < kept.mean() < 0.999  # both sides of the threshold are present
    rel = np.abs(dh - exact)[kept] / exact[kept]
    assert np.all(rel <= (1.0 / (rho - 1.0)) * (1 + 1e-6))
    # the paper's alpha (FP16/BF16 arithmetic throughout) is larger
    assert a < oracle.alpha_value(fmt, d, rho, "eq")
    # quantisation errors aligned with the differences (paired rows)
    Xa, Ca = _aligned_pairs(d, fmt, 50 + d + fmt)
    dha, Sa = _fp32_expanded(Xa, Ca, fmt)
    dha, Sa = np.diag(dha), np.diag(Sa)
    exa = np.diag(oracle.dist_rows(Xa, Ca))
    rela = np.abs(dha - exa) / exa
    keep_a = dha > a * Sa
    assert np.all(rela[keep_a] <= (1.0 / (rho - 1.0)) * (1 + 1e-6))
    # a planted mistake: without the conversion term the threshold keeps
    # aligned pairs whose quantisation error exceeds the bound (where the
    # FP32 arithmetic term alone is small enough for this to happen)
    if fmt == oracle.BF16 or d <= 8:
        assert np.any(rela[dha > a_bad * Sa] > 1.0 / (rho - 1.0))


def test_hw_alpha_cancellation_all_flagged():
    # every coordinate near 1e3 with spread 1e-2: the conversion error alone
    # exceeds the distances, so the hardware-aware test flags every pair
    X, C = W.cancellation_pair(200, 16, 64, seed=41)
    for fmt in (oracle.FP16, oracle.BF16):
        dh, S = _fp32_expanded(X, C, fmt)
        a = oracle.alpha_value(fmt, 64, 5.0, "hw")
        assert np.all(dh <= a * S)


# ---------------------------------------------------------------------------
# O4's bound A on the FP32 evaluation of the expanded formula
# ---------------------------------------------------------------------------

def _lib_round(a, fmt):
    """Rounded inputs from library conversions (numpy float16, torch
    bfloat16), as float32: independent of the oracle's own rounding."""
    if fmt == oracle.FP16:
        return a.astype(np.float16).astype(np.float32)
    torch = pytest.importorskip("torch")
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.bfloat16).float().numpy()


def _f32_sum_seq(terms):
    """Sequential float32 sum over the last axis (one rounding per add)."""
    acc = np.zeros(terms.shape[:-1], dtype=np.float32)
    for l in range(terms.shape[-1]):
        acc = (acc + terms[..., l]).astype(np.float32)
    return acc


def _f32_sum_pairwise(terms):
    t = terms.astype(np.float32)
    while t.shape[-1] > 1:
        if t.shape[-1] % 2:
            t = np.concatenate([t, np.zeros(t.shape[:-1] + (1,), np.float32)], axis=-1)
        t = (t[..., 0::2] + t[..., 1::2]).astype(np.float32)
    return t[..., 0]


def _f32_sum_blocked(terms, width, init=None):
    """Blocks of `width` consecutive terms summed exactly (FP64 holds the sum
    of a few products of 11- or 8-bit significands without loss at these
    magnitudes) and rounded once, then accumulated in float32 -- the shape of
    a matrix-core K step."""
    acc = np.zeros(terms.shape[:-1], dtype=np.float32) if init is None else init.astype(np.float32)
    for s in range(0, terms.shape[-1], width):
        blk = terms[..., s:s + width].astype(np.float64).sum(axis=-1).astype(np.float32)
        acc = (acc + blk).astype(np.float32)
    return acc


def _expanded_fp32_variants(Xq, Cq):
    """d^ = max(||x~||^2 + ||c~||^2 - 2 x~^T c~, 0) in float32 under several
    summation orders, including the accumulator form W = -||c~||^2/2 +
    x~^T c~, d^ = ||x~||^2 - 2W.  Products of FP16/BF16 values are exact in
    float32.  Returns a list of (name, (m, k) float64 arrays)."""
    prod = Xq[:, None, :] * Cq[None, :, :]  # exact float32 products
    sqx = Xq * Xq
    sqc = Cq * Cq
    out = []
    for name, red in (("sequential", _f32_sum_seq), ("pairwise", _f32_sum_pairwise),
                      ("blocked16", lambda t: _f32_sum_blocked(t, 16)),
                      ("blocked8", lambda t: _f32_sum_blocked(t, 8)),
                      ("reversed", lambda t: _f32_sum_seq(t[..., ::-1]))):
        nx = red(sqx)[:, None]
        nc = red(sqc)[None, :]
        dot = red(prod)
        dh = ((nx + nc).astype(np.float32) - (np.float32(2) * dot).astype(np.float32)).astype(np.float32)
        out.append((name, np.maximum(dh, np.float32(0)).astype(np.float64)))
    # accumulator form: start at -||c~||^2/2, add the K steps, d^ = nx - 2W
    nx = _f32_sum_blocked(sqx, 8)[:, None]
    nc = _f32_sum_seq(sqc)[None, :]
    W = _f32_sum_blocked(prod, 16, init=np.broadcast_to(-np.float32(0.5) * nc, prod.shape[:2]))
    dh = (nx - (np.float32(2) * W).astype(np.float32)).astype(np.float32)
    out.append(("accumulator", np.maximum(dh, np.float32(0)).astype(np.float64)))
    return out


def _aligned_rows(rows, d, g, p=7):
    # p = 7 fraction bits: representable in BF16 and FP16 alike
    v = np.empty((rows, d), dtype=np.float32)
    v[:, 0] = 2048.0
    v[:, 1:] = 0.5 * (1.0 + 2.0 ** -p) * np.where(g.random((rows, d - 1)) < 0.5, -1.0, 1.0)
    return v


def _a_cases(d, seed):
    g = np.random.default_rng(seed)
    m, k = 48, 64
    yield "normal", (g.standard_normal((m, d)).astype(np.float32),
                     g.standard_normal((k, d)).astype(np.float32))
    yield "cancellation", ((1e3 + 1e-2 * g.standard_normal((m, d))).astype(np.float32),
                           (1e3 + 1e-2 * g.standard_normal((k, d))).astype(np.float32))
    # every coordinate positive and of similar size: rounding errors of the
    # sums share a sign, and x~^T c~ is close to its bound ||x~|| ||c~||
    yield "sign_aligned", (g.uniform(0.5, 1.5, (m, d)).astype(np.float32),
                           g.uniform(0.5, 1.5, (k, d)).astype(np.float32))
    # mixed magnitudes: large and tiny coordinates in one row
    scale = 10.0 ** g.integers(-3, 3, size=d)
    yield "mixed_scale", ((g.standard_normal((m, d)) * scale).astype(np.float32),
                          (g.standard_normal((k, d)) * scale).astype(np.float32))
    # rounding-aligned sums: a leading coordinate 2048 (square 2^22, FP32
    # spacing 1/2 there) followed by coordinates +-(1/2)(1 + 2^-p), whose
    # squares exceed a quarter by a little, so that every addition of a
    # sequential FP32 sum of squares rounds up by almost half a spacing
    yield "rounding_aligned", (_aligned_rows(m, d, g), _aligned_rows(k, d, g))


@pytest.mark.parametrize("fmt", [oracle.FP16, oracle.BF16])
@pytest.mark.parametrize("d", [5, 64, 128])
def test_mp_bound_A_covers_fp32_evaluations(fmt, d):
    # Theorem thm:dist-exp applied to the rounded inputs with FP32
    # arithmetic: every FP32 evaluation of the expanded formula of x~, c~
    # lies within A = gamma'_{d+4}(S + 2|x~|^T|c~|) of q = d(x~, c~)^2,
    # whatever the summation order.  The evaluations here are written
    # independently of the oracle (library rounding, numpy float32).
    worst = 0.0
    for case, (X, C) in _a_cases(d, 700 + 10 * d + fmt):
        if fmt == oracle.FP16 and case == "mixed_scale":
            X = np.clip(X, -6e4, 6e4)
            C = np.clip(C, -6e4, 6e4)
        r = oracle.mp_rows(X, C, fmt, 0.5)
        assert r["n_bad"] == 0
        Xq, Cq = _lib_round(X, fmt), _lib_round(C, fmt)
        P = np.abs(Xq.astype(np.float64)) @ np.abs(Cq.astype(np.float64)).T
        for name, dh in _expanded_fp32_variants(Xq, Cq):
            err = np.abs(dh - r["q"])
            assert np.all(err <= r["A"]), "%s/%s: FP32 error %.3g exceeds A %.3g" % (
                case, name, err.max(), r["A"].flat[np.argmax(err - r["A"])])
            worst = max(worst, float((err / r["A"]).max()))
            # a planted slip: A built on the FP64 unit roundoff instead of
            # twice the FP32 one is far too small for any FP32 evaluation
            A_slip = oracle.gamma(d + 4, oracle.unit_roundoff(3)) * (r["S"] + 2 * P)
            if np.any(err > 0):
                assert np.any(err > A_slip), "%s/%s: slip not detected" % (case, name)
            if case == "rounding_aligned" and name == "sequential" and d >= 64:
                # another planted slip: the length of the sum dropped from
                # the bound (gamma'_4 instead of gamma'_{d+4})
                A_short = oracle.gamma(4, 2 * oracle.unit_roundoff(2)) * (r["S"] + 2 * P)
                assert np.any(err > A_short), "dropped dimension not detected"
    # the bound is not vacuous: some evaluation uses a visible part of it
    assert worst > 1e-4, "largest error only %.3g of A" % worst


@pytest.mark.parametrize("fmt", [oracle.FP16, oracle.BF16])
def test_mp_classes_bracket_fp32_test_decisions(fmt):
    # the band of O4's classes covers the FP32 evaluation of the test in the
    # accumulator form (flag iff W + alpha nc/2 >= (1 - alpha) nx / 2): a
    # surely corrected pair is flagged and a surely kept one is not, for
    # every summation order of the cross term
    d = 32
    X, C = _boundary_pairs(d, 90 + fmt)
    a = np.float32(0.25)
    r = oracle.mp_rows(X, C, fmt, float(a))
    Xq, Cq = _lib_round(X, fmt), _lib_round(C, fmt)
    prod = Xq[:, None, :] * Cq[None, :, :]
    nx = _f32_sum_blocked(Xq * Xq, 8)
    nc = _f32_sum_seq(Cq * Cq)
    hx = (np.float32(0.5) * ((np.float32(1) - a) * nx).astype(np.float32)).astype(np.float32)
    ca = (a * (np.float32(0.5) * nc).astype(np.float32)).astype(np.float32)
    init = np.broadcast_to(-(np.float32(0.5) * nc), prod.shape[:2])
    for W in (_f32_sum_blocked(prod, 16, init=init),
              (init + _f32_sum_seq(prod)).astype(np.float32)):
        flag = (W + ca[None, :]).astype(np.float32) >= hx[:, None]
        assert np.all(flag[r["cls"] == -1])
        assert not np.any(flag[r["cls"] == 1])
    # both classes occur, and the ambiguous band is a small minority
    assert (r["cls"] == -1).any() and (r["cls"] == 1).any()
    assert (r["cls"] == 0).mean() < 0.05
