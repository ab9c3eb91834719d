"""Shared checks for the GPU parity tests (host side only).

The checks compare what the HIP library returned with the CPU oracle on the
same float32 inputs, following the parity contract:

  (i)   label gate: where the oracle's best centre beats every other centre
        by more than the per-pair error bounds B, labels must be identical;
  (ii)  distances within relative 1e-6 of the oracle's FP64 direct value to
        the returned label, SSE within relative 1e-6, and near-optimality
        d(i, label) <= d(i, j1) + B(i, label) + B(i, j1) everywhere;
  (iii) the number of corrected pairs lies between the count of surely
        corrected pairs and that count plus the ambiguous ones.
"""

import numpy as np

import oracle

DIST_RTOL = 1e-6


def fp32_classes(Xs, C, alpha, dist):
    """Per-pair classification for FP32 operands (quantisation is the
    identity, so the oracle's O4 rounding does not apply): the FP32 bound A
    of Theorem thm:dist-exp, the margin of the test against a band of
    (1 + alpha) A plus the FP64 value's own rounding, and the error bound B
    of the value the GPU reports.  Returns (cls, B): -1 surely flagged,
    +1 surely kept, 0 ambiguous."""
    u32 = oracle.unit_roundoff(2)
    xn = (Xs.astype(np.float64) ** 2).sum(1)[:, None]
    cn = (C.astype(np.float64) ** 2).sum(1)[None, :]
    P = np.abs(Xs.astype(np.float64)) @ np.abs(C.astype(np.float64)).T
    g = oracle.gamma(Xs.shape[1] + 4, 2 * u32)
    A = g * (xn + cn + 2 * P)
    B = A + 2 * u32 * dist
    S = xn + cn
    if alpha is None or alpha < 0:
        return np.ones(dist.shape, dtype=np.int8), B
    margin = dist - alpha * S
    band = (1 + alpha) * A + 2 * u32 * dist
    cls = np.where(margin < -band, -1, np.where(margin > band, 1, 0)).astype(np.int8)
    B = np.where(cls == -1, 2 * u32 * dist, np.where(cls == 1, B, np.maximum(B, 2 * u32 * dist)))
    return cls, B


def check_assignment(X, C, fmt, alpha, labels, mindist, sse, n_corrected,
                     min_coverage=0.0, rows=None, check_sandwich=True):
    """Apply (i)-(iii).  ``rows`` restricts the check to a subset of points
    (the GPU outputs are then full-length and are indexed by ``rows``).
    ``fmt`` is 0 (FP16) / 1 (BF16) / 2 (FP32: quantisation is the identity)
    / None (plain FP64 direct formula everywhere).  Returns a report dict."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    C = np.ascontiguousarray(C, dtype=np.float32)
    if rows is None:
        rows = np.arange(X.shape[0])
    Xs = X[rows]
    lab = np.asarray(labels)[rows].astype(np.int64)
    if fmt in (0, 1):
        r = oracle.mp_rows(Xs, C, fmt, alpha)
        dist, B, cls = r["dist"], r["B"], r["cls"]
    else:
        dist = oracle.dist_rows(Xs, C)
        u32 = oracle.unit_roundoff(2)
        if fmt is None:  # FP64 direct everywhere, compared in FP64
            B = 2 * oracle.gamma(X.shape[1] + 2, oracle.unit_roundoff(3)) * dist
            cls = np.full(dist.shape, -1, dtype=np.int8)
        else:  # FP32 expanded formula: error bound of thm:dist-exp in FP32
            cls, B = fp32_classes(Xs, C, alpha, dist)
    m = len(rows)
    ii = np.arange(m)
    j1 = np.argmin(dist, axis=1)  # lowest index among exact minimisers
    gated = oracle.label_gate(dist, B, j1)
    bad = np.nonzero(gated & (lab != j1))[0]
    assert bad.size == 0, "gated label mismatch at rows %s (gpu %s, oracle %s)" % (
        rows[bad[:5]], lab[bad[:5]], j1[bad[:5]])
    coverage = float(gated.mean())
    assert coverage >= min_coverage, "gate coverage %.4f < %.4f" % (coverage, min_coverage)
    d_lab = dist[ii, lab]
    # near-optimality of the returned label
    slack = dist[ii, j1] + B[ii, lab] + B[ii, j1]
    assert np.all(d_lab <= slack * (1 + 1e-12) + 1e-300), "label not near-optimal"
    if mindist is not None:
        md = np.asarray(mindist)[rows].astype(np.float64)
        err = np.abs(md - d_lab)
        tol = DIST_RTOL * d_lab + 1e-30
        worst = int(np.argmax(err - tol))
        assert np.all(err <= tol), "mindist off at row %d: %r vs %r" % (
            rows[worst], md[worst], d_lab[worst])
    rep = dict(coverage=coverage, n_rows=m)
    if sse is not None and len(rows) == X.shape[0]:
        ref = oracle.pairwise_sum(d_lab)
        assert abs(sse - ref) <= DIST_RTOL * abs(ref) + 1e-30, "SSE %r vs %r" % (sse, ref)
        rep["sse_ref"] = ref
    n_sure = int((cls == -1).sum())
    n_amb = int((cls == 0).sum())
    rep.update(n_sure=n_sure, n_amb=n_amb)
    if check_sandwich and n_corrected is not None and len(rows) == X.shape[0]:
        assert n_sure <= n_corrected <= n_sure + n_amb, \
            "corrected %d not in [%d, %d]" % (n_corrected, n_sure, n_sure + n_amb)
    return rep


def check_pairwise(X, C, fmt, alpha, D, flagged):
    """Per-pair checks on materialised values: flagged pairs are the FP64
    direct value rounded once to FP32; kept pairs are within A of the
    quantised distance q (Theorem thm:dist-exp with FP32 arithmetic, P10);
    surely corrected pairs are flagged and surely kept ones are not."""
    r = oracle.mp_rows(X, C, fmt, alpha)
    D = np.asarray(D, dtype=np.float64)
    fl = np.asarray(flagged).astype(bool)
    u32 = oracle.unit_roundoff(2)
    cls = r["cls"]
    assert not np.any(fl & (cls == 1)), "a surely kept pair was corrected"
    assert not np.any(~fl & (cls == -1)), "a surely corrected pair was kept"
    corr = fl
    err_c = np.abs(D[corr] - r["dist"][corr])
    assert np.all(err_c <= 2 * u32 * r["dist"][corr] + 1e-30), "corrected value off"
    kept = ~fl
    err_k = np.abs(D[kept] - r["q"][kept])
    # kept values are clamped at zero (max(d^, 0)); the bound covers that
    assert np.all(err_k <= r["A"][kept] * (1 + 1e-9) + 1e-30), \
        "kept pair outside the FP32 expanded-formula bound (max excess %.3g)" % (
            np.max(err_k - r["A"][kept]))
    rel = np.abs(D - r["dist"]) / np.maximum(r["dist"], 1e-300)
    return dict(n_flagged=int(fl.sum()), n_sure=int((cls == -1).sum()),
                n_amb=int((cls == 0).sum()), max_rel_err=float(rel.max()),
                max_rel_err_kept=float(rel[kept].max()) if kept.any() else 0.0)


def scan_rows(X, C, fmt, alpha, label_arrays):
    """O4 over every pair of X against C, streamed (oracle.mp_scan), with the
    oracle quantities at each of the given GPU label arrays."""
    return oracle.mp_scan(X, C, fmt, -1.0 if alpha is None else alpha, label_arrays)


def check_assignment_scan(scan, t, labels, mindist, sse, n_corrected, *, bound="mp",
                          d=None, min_coverage=0.0, check_sandwich=True):
    """(i)-(iii) over ALL rows from a streamed scan (``scan_rows``); ``t``
    selects which of the scan's label arrays ``labels`` is.  ``bound="mp"``
    applies O4's bounds (fmt and alpha of the scan); ``bound="fp64"`` the
    plain FP64 direct formula compared in FP64 (B = 2 gamma_{d+2}(u_64)
    dist, ``d`` required)."""
    lab = np.asarray(labels).astype(np.int64)
    j1 = scan["j1"].astype(np.int64)
    dj1 = scan["dj1"]
    d_lab = scan["dlab"][t]
    if bound == "fp64":
        g = 2 * oracle.gamma(d + 2, oracle.unit_roundoff(3))
        Bj1 = g * dj1
        Blab = g * d_lab
        gated = scan["d2"] * (1 - g) > dj1 * (1 + g)
    else:
        Bj1 = scan["Bj1"]
        Blab = scan["Blab"][t]
        gated = scan["lo"] > dj1 + Bj1
    assert np.all(np.isfinite(d_lab)), "label out of range"
    bad = np.nonzero(gated & (lab != j1))[0]
    assert bad.size == 0, "gated label mismatch at rows %s (gpu %s, oracle %s)" % (
        bad[:5], lab[bad[:5]], j1[bad[:5]])
    coverage = float(gated.mean())
    assert coverage >= min_coverage, "gate coverage %.5f < %.5f" % (coverage, min_coverage)
    slack = dj1 + Blab + Bj1
    far = np.nonzero(d_lab > slack * (1 + 1e-12) + 1e-300)[0]
    assert far.size == 0, "label not near-optimal at rows %s" % far[:5]
    rep = dict(coverage=coverage, n_rows=len(lab), n_ungated=int((~gated).sum()),
               n_diff=int((lab != j1).sum()))
    if mindist is not None:
        md = np.asarray(mindist).astype(np.float64)
        err = np.abs(md - d_lab)
        tol = DIST_RTOL * d_lab + 1e-30
        worst = int(np.argmax(err - tol))
        assert np.all(err <= tol), "mindist off at row %d: %r vs %r" % (worst, md[worst], d_lab[worst])
    if sse is not None:
        ref = oracle.pairwise_sum(d_lab)
        assert abs(sse - ref) <= DIST_RTOL * abs(ref) + 1e-30, "SSE %r vs %r" % (sse, ref)
        rep["sse_ref"] = ref
        rep["sse_rel_err"] = abs(sse - ref) / abs(ref)
    c = scan["counts"]
    rep.update(n_sure=int(c[0]), n_amb=int(c[1]))
    if check_sandwich and n_corrected is not None and bound == "mp":
        assert c[0] <= n_corrected <= c[0] + c[1], \
            "corrected %d not in [%d, %d]" % (n_corrected, c[0], c[0] + c[1])
    return rep


def corr_intervals(X, C, fmt, alpha, high):
    """Per pair, the interval the value a GPU pass compares may take under
    correction precision ``high`` (0 FP64, 1 FP32, 2 the low format): a
    surely corrected pair takes exactly O5's value (FP64 rounded once to
    FP32; FP32 and low-format values are FP32 numbers), a surely kept pair
    lies within O4's bound A of the quantised distance q (FP16/BF16) or
    within A + 2 u_32 dist of dist (FP32 inputs), an ambiguous pair may take
    either.  Returns (lo, hi, cls, h32, dist)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    C = np.ascontiguousarray(C, dtype=np.float32)
    h32 = oracle.corr_rows(X, C, high, fmt).astype(np.float32).astype(np.float64)
    if fmt in (0, 1):
        r = oracle.mp_rows(X, C, fmt, alpha)
        dist, cls = r["dist"], r["cls"]
        klo = r["q"] - r["A"] * (1 + 1e-9) - 1e-30
        khi = r["q"] + r["A"] * (1 + 1e-9) + 1e-30
    else:
        dist = oracle.dist_rows(X, C)
        u32 = oracle.unit_roundoff(2)
        xn = (X.astype(np.float64) ** 2).sum(1)[:, None]
        cn = (C.astype(np.float64) ** 2).sum(1)[None, :]
        P = np.abs(X.astype(np.float64)) @ np.abs(C.astype(np.float64)).T
        A = oracle.gamma(X.shape[1] + 4, 2 * u32) * (xn + cn + 2 * P)
        Bk = A + 2 * u32 * dist
        klo, khi = dist - Bk, dist + Bk
        margin = dist - alpha * (xn + cn)
        band = (1 + alpha) * A + 2 * u32 * dist
        cls = np.where(margin < -band, -1, np.where(margin > band, 1, 0)).astype(np.int8)
    klo = np.maximum(klo, 0.0)  # kept values are clamped at zero
    lo = np.where(cls == -1, h32, np.where(cls == 1, klo, np.minimum(h32, klo)))
    hi = np.where(cls == -1, h32, np.where(cls == 1, khi, np.maximum(h32, khi)))
    return lo, hi, cls, h32, dist


def check_assignment_high(X, C, fmt, alpha, high, labels, mindist, n_corrected, min_coverage=0.0):
    """Labels of a pass with correction precision ``high``: the returned label
    can be a minimiser of the compared values (its interval starts at or
    below the smallest interval end of the row), equals the only such centre
    where there is one, and is the lowest index when every candidate is a
    corrected pair of the same value.  mindist is the FP64 refinement of the
    returned label; the corrected-pair count lies between the surely
    corrected and the surely corrected plus ambiguous pairs."""
    lo, hi, cls, h32, dist = corr_intervals(X, C, fmt, alpha, high)
    lab = np.asarray(labels).astype(np.int64)
    m = lo.shape[0]
    ii = np.arange(m)
    H = hi.min(axis=1)
    cand = lo <= H[:, None]
    assert np.all(cand[ii, lab]), "label not a possible minimiser at rows %s" % (
        np.nonzero(~cand[ii, lab])[0][:5])
    ncand = cand.sum(axis=1)
    single = ncand == 1
    first = np.argmax(cand, axis=1)
    assert np.all(lab[single] == first[single])
    pts = np.all(~cand | ((cls == -1) & (h32 == H[:, None])), axis=1) & ~single
    assert np.all(lab[pts] == first[pts]), "tie of corrected values not resolved to the lowest index"
    coverage = float(single.mean())
    assert coverage >= min_coverage, "gate coverage %.4f < %.4f" % (coverage, min_coverage)
    if mindist is not None:
        md = np.asarray(mindist).astype(np.float64)
        d_lab = dist[ii, lab]
        assert np.all(np.abs(md - d_lab) <= DIST_RTOL * d_lab + 1e-30), "mindist is not the FP64 value"
    n_sure, n_amb = int((cls == -1).sum()), int((cls == 0).sum())
    if n_corrected is not None:
        assert n_sure <= n_corrected <= n_sure + n_amb, \
            "corrected %d not in [%d, %d]" % (n_corrected, n_sure, n_sure + n_amb)
    return dict(coverage=coverage, ties=int(pts.sum()), n_sure=n_sure, n_amb=n_amb)
