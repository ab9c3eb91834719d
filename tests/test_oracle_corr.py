"""Pins of O5 (oracle/kmeans_oracle.c): the value of a flagged pair under
another fallback precision (eq:fallback-rule, eq:fallback-rule-mp; the
variants of Section 6.1).  The rounding of exact results is checked against
two independent definitions: nearest value by enumeration of every finite
binary16 / bfloat16 number (ties to the even bit pattern), and, for binary32,
exact rational arithmetic on the format's grid.  CPU only."""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

# (significand bits t, emin, emax) of Table table:float-arith-parameter
FMTS = {0: (11, -14, 15), 1: (8, -126, 127), 2: (24, -126, 127)}


def _all_values(fmt):
    """Every finite non-negative value of binary16 (fmt 0) or bfloat16
    (fmt 1), ascending, with its bit pattern."""
    bits = np.arange(0, 0x7c00 if fmt == 0 else 0x7f80, dtype=np.uint32)
    if fmt == 0:
        vals = bits.astype(np.uint16).view(np.float16).astype(np.float64)
    else:
        vals = (bits << 16).view(np.float32).astype(np.float64)
    return vals, bits


_TABLES = {}


def rne_table(v: Fraction, fmt: int) -> float:
    """Nearest binary16/bfloat16 value to v, ties to the even bit pattern, by
    enumeration of the format; beyond the largest finite value the next
    pattern is infinity (even), as IEEE 754 overflow does."""
    if fmt not in _TABLES:
        _TABLES[fmt] = _all_values(fmt)
    vals, bits = _TABLES[fmt]
    a = abs(v)
    i = int(np.searchsorted(vals, float(a)))
    cands = []
    for j in (i - 2, i - 1, i, i + 1):
        if 0 <= j < len(vals):
            cands.append((Fraction(vals[j]), int(bits[j])))
    t, _, emax = FMTS[fmt]
    top = Fraction(2) ** (emax + 1)
    cands.append((top, int(bits[-1]) + 1))  # infinity's pattern (even)
    best = min(cands, key=lambda c: (abs(c[0] - a), c[1] & 1))
    r = math.inf if best[0] == top else float(best[0])
    return -r if v < 0 else r


def rne_grid(v: Fraction, fmt: int) -> float:
    """Nearest value of the format to v on its grid, ties to even, in exact
    rational arithmetic (the binade 2^e <= |v| < 2^(e+1), e >= emin, has
    spacing 2^(e+1-t))."""
    t, emin, emax = FMTS[fmt]
    if v == 0:
        return 0.0
    a = abs(v)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    sp = Fraction(2) ** (e + 1 - t)
    q = a / sp
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    r = n * sp
    if r > (2 - Fraction(2) ** (1 - t)) * Fraction(2) ** emax:
        return -math.inf if v < 0 else math.inf
    return float(-r if v < 0 else r)


def rne(v, fmt):
    return rne_table(v, fmt) if fmt in (0, 1) else rne_grid(v, fmt)


def _random_values(fmt, count, rng, lo_exp, hi_exp):
    """Random values of the format: random significands, exponents in
    [lo_exp, hi_exp], random signs (some exact zeros)."""
    t, emin, _ = FMTS[fmt]
    e = rng.integers(lo_exp, hi_exp + 1, size=count)
    m = rng.integers(0, 2 ** (t - 1), size=count)
    v = [rne_grid(Fraction(2 ** (t - 1) + int(mi), 2 ** (t - 1)) * Fraction(2) ** int(ei), fmt)
         for mi, ei in zip(m, e)]
    s = rng.choice([-1.0, 1.0], size=count)
    v = np.array(v) * s
    v[rng.random(count) < 0.02] = 0.0
    return v


def test_enumeration_and_grid_agree():
    # the two independent definitions agree on binary16 and bfloat16
    rng = np.random.default_rng(1)
    for fmt in (0, 1):
        for _ in range(400):
            v = Fraction(float(rng.standard_normal())) * Fraction(2) ** int(rng.integers(-30, 20))
            assert rne_table(v, fmt) == rne_grid(v, fmt)


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_low_sub_and_fma_round_once(fmt):
    rng = np.random.default_rng(10 + fmt)
    t, emin, emax = FMTS[fmt]
    # exponents spanning subnormal results and near-overflow products
    lo, hi = (emin - 3, emax // 2) if fmt else (-24, 7)
    a = _random_values(fmt, 600, rng, lo, hi)
    b = _random_values(fmt, 600, rng, lo, hi)
    c = _random_values(fmt, 600, rng, lo, hi)
    for x, y, z in zip(a, b, c):
        assert oracle.low_sub(x, y, fmt) == rne(Fraction(x) - Fraction(y), fmt), (fmt, x, y)
        assert oracle.low_fma(x, y, z, fmt) == rne(Fraction(x) * Fraction(y) + Fraction(z), fmt), (fmt, x, y, z)


@pytest.mark.parametrize("fmt,step", [(0, 2.0 ** -10), (1, 2.0 ** -7), (2, 2.0 ** -23)])
def test_fma_ties_and_inexact_fp64_sums(fmt, step):
    # 1.5 * (1 + step) = 1.5 + step + step/2 lies halfway between two
    # neighbours (spacing `step` near 1.5): ties to even, unless an addend
    # pushes it; for bfloat16 and binary32 an addend of 2^-100 / 2^-120 makes
    # the FP64 sum inexact, and only its error term decides
    a, b = 1.5, 1.0 + step
    even = 1.5 + 2 * step  # ...10 (even) rather than ...01
    assert oracle.low_fma(a, b, 0.0, fmt) == even
    tiny = {0: 2.0 ** -24, 1: 2.0 ** -100, 2: 2.0 ** -120}[fmt]
    assert oracle.low_fma(a, b, tiny, fmt) == 1.5 + 2 * step
    assert oracle.low_fma(a, b, -tiny, fmt) == 1.5 + step
    for z in (0.0, tiny, -tiny):
        assert oracle.low_fma(a, b, z, fmt) == rne(Fraction(a) * Fraction(b) + Fraction(z), fmt)


def test_round_exact_overflow_and_subnormals():
    # binary16: 65520 is halfway between 65504 and 2^16 and goes to infinity
    assert oracle.round_exact(65520.0, 0.0, 0) == math.inf
    assert oracle.round_exact(65520.0, -1e-30, 0) == 65504.0
    # smallest binary16 subnormal 2^-24; half of it ties to zero (even)
    assert oracle.round_exact(2.0 ** -25, 0.0, 0) == 0.0
    assert oracle.round_exact(2.0 ** -25, 1e-40, 0) == 2.0 ** -24
    assert oracle.round_exact(3 * 2.0 ** -25, 0.0, 0) == 2.0 ** -23
    # bfloat16 keeps binary32's exponent range
    assert oracle.round_exact(2.0 ** -133, 0.0, 1) == 2.0 ** -133
    assert oracle.round_exact(-2.0 ** -134, 0.0, 1) == -0.0


def _corr_by_primitives(x, c, high, fmt):
    f = 2 if high == 1 else fmt
    s = 0.0
    for xv, cv in zip(x, c):
        if high == 2 and fmt != 2:
            xv, cv = oracle.round_low(np.float32(xv), fmt), oracle.round_low(np.float32(cv), fmt)
        t = rne(Fraction(float(xv)) - Fraction(float(cv)), f)
        s = rne(Fraction(t) * Fraction(t) + Fraction(s), f)
    return s


@pytest.mark.parametrize("high,fmt", [(1, 0), (1, 1), (2, 0), (2, 1), (2, 2)])
def test_corr_rows_compose_the_rounded_operations(high, fmt):
    rng = np.random.default_rng(3 + 7 * high + fmt)
    X = (rng.standard_normal((6, 9)) * 4).astype(np.float32)
    C = (rng.standard_normal((5, 9)) * 4).astype(np.float32)
    X[0] = C[1] + np.float32(1e-3)  # a near pair
    H = oracle.corr_rows(X, C, high, fmt)
    for i in range(X.shape[0]):
        for j in range(C.shape[0]):
            assert H[i, j] == _corr_by_primitives(X[i], C[j], high, fmt), (i, j)
    # FP64 fallback is O1's sum
    np.testing.assert_array_equal(oracle.corr_rows(X, C, 0, fmt), oracle.dist_rows(X, C))


def test_uniform_fallback_loses_the_true_difference():
    # 1 and 1 + 2^-12 are one binary16 number apart only after rounding: the
    # uniform FP16 fallback sees two equal operands, the FP32 and FP64
    # fallbacks the true distance 2^-24 (exact in both)
    x = np.array([[1.0]], dtype=np.float32)
    c = np.array([[1.0 + 2.0 ** -12]], dtype=np.float32)
    assert oracle.corr_rows(x, c, 2, 0)[0, 0] == 0.0
    assert oracle.corr_rows(x, c, 1, 0)[0, 0] == 2.0 ** -24
    assert oracle.corr_rows(x, c, 0, 0)[0, 0] == 2.0 ** -24
    # bfloat16 (8 bits): 1 + 2^-9 rounds to 1 as well
    c2 = np.array([[1.0 + 2.0 ** -9]], dtype=np.float32)
    assert oracle.corr_rows(x, c2, 2, 1)[0, 0] == 0.0
    # binary16 overflow of the running sum
    big = np.array([[200.0, 200.0]], dtype=np.float32)
    assert oracle.corr_rows(big, -big, 2, 0)[0, 0] == math.inf


# ---------------------------------------------------------------------------
# O6: k-means++ seeding by D^2 weighting
# ---------------------------------------------------------------------------

def test_seed_pp_worked_example_on_a_line():
    # points 0, 1, 3, 10 on a line; first seed floor(0.3 * 4) = 1 (x = 1);
    # weights to it: 1, 0, 4, 81 (total 86): u = 0.5 -> 43 falls in the last
    # point's share; then weights 1, 0, 4, 0 (total 5): u = 0.3 -> 1.5 falls
    # in point 2's share (1 < 1.5 <= 5)
    X = np.array([[0.0], [1.0], [3.0], [10.0]], dtype=np.float32)
    assert list(oracle.seed_pp(X, 3, [0.3, 0.5, 0.3])) == [1, 3, 2]
    # u = 0 picks the first point of positive weight; a weight of zero is
    # never picked, however u falls
    assert list(oracle.seed_pp(X, 2, [0.3, 0.0])) == [1, 0]


def test_seed_pp_draws_points_in_proportion_to_d2():
    # with the first seed fixed, the second is point p with probability
    # w_p / sum(w): the frequencies over a fine grid of u equal the shares
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0], [3.0, 4.0], [-1.0, -1.0]], dtype=np.float32)
    w = ((X - X[0]) ** 2).sum(1).astype(np.float64)
    grid = (np.arange(20000) + 0.5) / 20000
    counts = np.zeros(5)
    for u in grid:
        counts[oracle.seed_pp(X, 2, [0.0, u])[1]] += 1
    np.testing.assert_allclose(counts / len(grid), w / w.sum(), atol=1e-4)


def test_seed_pp_degenerate_and_distinct():
    X = np.ones((6, 3), dtype=np.float32)  # all points coincide
    assert list(oracle.seed_pp(X, 3, [0.0, 0.5, 0.99])) == [0, 3, 5]
    g = np.random.default_rng(2)
    Y = g.standard_normal((500, 4)).astype(np.float32)
    idx = oracle.seed_pp(Y, 50, g.random(50))
    assert len(set(idx.tolist())) == 50  # distinct points are never drawn twice
