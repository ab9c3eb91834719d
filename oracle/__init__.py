"""CPU oracle for mixed-precision Lloyd k-means -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
it shares no code with the GPU path; both receive the same float32 arrays from
the ``workloads`` module.

The arithmetic lives in ``kmeans_oracle.c`` (plain C, FP64, OpenMP over
points); this module compiles it with gcc and marshals numpy arrays through
ctypes.  See the C file for what each function computes and which passage of
the paper it follows.
"""

from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kmeans_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lock = threading.Lock()
_lib = None

FP16, BF16, FP32, FP64 = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE semantics: no fast-math, no FMA
    contraction)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if not force and os.path.exists(_LIB) and \
            os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or \
                    os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ct.CDLL(_LIB)
            P = ct.c_void_p
            i64, i32, dbl = ct.c_int64, ct.c_int, ct.c_double
            L.oracle_unit_roundoff.restype = dbl
            L.oracle_unit_roundoff.argtypes = [i32]
            L.oracle_fmt_max.restype = dbl
            L.oracle_fmt_max.argtypes = [i32]
            L.oracle_fmt_min_normal.restype = dbl
            L.oracle_fmt_min_normal.argtypes = [i32]
            L.oracle_fmt_params.restype = i32
            L.oracle_fmt_params.argtypes = [i32, P, P, P]
            L.oracle_gamma.restype = dbl
            L.oracle_gamma.argtypes = [dbl, dbl]
            L.oracle_round_low.restype = dbl
            L.oracle_round_low.argtypes = [ct.c_float, i32]
            L.oracle_quantize.restype = None
            L.oracle_quantize.argtypes = [P, i64, i32, P]
            L.oracle_round_exact.restype = dbl
            L.oracle_round_exact.argtypes = [dbl, dbl, i32]
            L.oracle_low_sub.restype = dbl
            L.oracle_low_sub.argtypes = [dbl, dbl, i32]
            L.oracle_low_fma.restype = dbl
            L.oracle_low_fma.argtypes = [dbl, dbl, dbl, i32]
            L.oracle_corr_dist.restype = dbl
            L.oracle_corr_dist.argtypes = [P, P, i32, i32, i32]
            L.oracle_seed_pp.restype = None
            L.oracle_seed_pp.argtypes = [P, i64, i32, i32, P, P]
            L.oracle_corr_rows.restype = None
            L.oracle_corr_rows.argtypes = [P, i64, i32, P, i32, i32, i32, P]
            L.oracle_sqdist.restype = dbl
            L.oracle_sqdist.argtypes = [P, P, i32]
            L.oracle_pairwise_sum.restype = dbl
            L.oracle_pairwise_sum.argtypes = [P, i64]
            L.oracle_dist_rows.restype = None
            L.oracle_dist_rows.argtypes = [P, i64, i32, P, i32, P]
            L.oracle_assign.restype = None
            L.oracle_assign.argtypes = [P, i64, i32, P, i32, P, P, P]
            L.oracle_sse_labels.restype = dbl
            L.oracle_sse_labels.argtypes = [P, i64, i32, P, P, i32]
            L.oracle_update.restype = i64
            L.oracle_update.argtypes = [P, i64, i32, P, i32, P, P, P, P]
            L.oracle_lloyd.restype = i32
            L.oracle_lloyd.argtypes = [P, i64, i32, i32, P, i32, dbl, P, P, P, P]
            L.oracle_mp_rows.restype = i64
            L.oracle_mp_rows.argtypes = [P, i64, i32, P, i32, i32, dbl,
                                         P, P, P, P, P, P]
            L.oracle_mp_scan.restype = i32
            L.oracle_mp_scan.argtypes = [P, i64, i32, P, i32, i32, dbl, i32, P,
                                         P, P, P, P, P, P, P, P]
            L.oracle_mp_count.restype = None
            L.oracle_mp_count.argtypes = [P, i64, i32, P, i32, i32, dbl, P]
            L.oracle_num_threads.restype = i32
            L.oracle_num_threads.argtypes = []
            L.oracle_set_num_threads.restype = None
            L.oracle_set_num_threads.argtypes = [i32]
            _lib = L
    return _lib


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


# ---------------------------------------------------------------------------
# Formats and constants (Table table:float-arith-parameter)
# ---------------------------------------------------------------------------

def unit_roundoff(fmt: int) -> float:
    return lib().oracle_unit_roundoff(fmt)


def fmt_max(fmt: int) -> float:
    return lib().oracle_fmt_max(fmt)


def fmt_min_normal(fmt: int) -> float:
    return lib().oracle_fmt_min_normal(fmt)


def fmt_params(fmt: int):
    t, emin, emax = ct.c_int(), ct.c_int(), ct.c_int()
    rc = lib().oracle_fmt_params(fmt, ct.byref(t), ct.byref(emin), ct.byref(emax))
    if rc != 0:
        raise ValueError(fmt)
    return t.value, emin.value, emax.value


def gamma(m: float, u: float) -> float:
    return lib().oracle_gamma(float(m), float(u))


def round_low(x, fmt: int) -> np.ndarray:
    """Round float32 values to FP16 (fmt 0) or BF16 (fmt 1), RNE; float64 out."""
    a = _f32(np.atleast_1d(x)).ravel()
    out = np.empty(a.shape[0], dtype=np.float64)
    lib().oracle_quantize(_ptr(a), a.shape[0], fmt, _ptr(out))
    return out.reshape(np.shape(x))


# ---------------------------------------------------------------------------
# O1 - O3
# ---------------------------------------------------------------------------

def sqdist(x, y) -> float:
    x, y = _f32(x), _f32(y)
    return lib().oracle_sqdist(_ptr(x), _ptr(y), x.shape[0])


def pairwise_sum(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().oracle_pairwise_sum(_ptr(v), v.shape[0])


def dist_rows(X, C) -> np.ndarray:
    X, C = _f32(X), _f32(C)
    m, d = X.shape
    k = C.shape[0]
    D = np.empty((m, k), dtype=np.float64)
    lib().oracle_dist_rows(_ptr(X), m, d, _ptr(C), k, _ptr(D))
    return D


def assign(X, C):
    """O1: labels (int32), FP64 distance to the label, SSE."""
    X, C = _f32(X), _f32(C)
    n, d = X.shape
    k = C.shape[0]
    labels = np.empty(n, dtype=np.int32)
    mind = np.empty(n, dtype=np.float64)
    sse = ct.c_double()
    lib().oracle_assign(_ptr(X), n, d, _ptr(C), k, _ptr(labels), _ptr(mind),
                        ct.byref(sse))
    return labels, mind, sse.value


def sse_labels(X, C, labels) -> float:
    """eq:sse of a given assignment: sum_i ||x_i - c_{labels_i}||^2, each
    term by the FP64 direct formula, pairwise summed (O1's order)."""
    X, C = _f32(X), _f32(C)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    v = lib().oracle_sse_labels(_ptr(X), X.shape[0], X.shape[1], _ptr(labels), _ptr(C), C.shape[0])
    if v < 0:
        raise ValueError("label out of range")
    return v


def update(X, labels, C_old):
    """O2: new centres (float32), counts, max shift, number of empty clusters."""
    X, C_old = _f32(X), _f32(C_old)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    n, d = X.shape
    k = C_old.shape[0]
    C_new = np.empty_like(C_old)
    counts = np.empty(k, dtype=np.int64)
    shift = ct.c_double()
    empty = lib().oracle_update(_ptr(X), n, d, _ptr(labels), k, _ptr(C_old),
                                _ptr(C_new), _ptr(counts), ct.byref(shift))
    if empty < 0:
        raise ValueError("label out of range")
    return C_new, counts, shift.value, int(empty)


def lloyd(X, C0, max_iter: int, tol: float = 0.0):
    """O3: returns dict(C, labels, mind, sse_hist, shift_hist, iters)."""
    X = _f32(X)
    C = _f32(C0).copy()
    n, d = X.shape
    k = C.shape[0]
    labels = np.empty(n, dtype=np.int32)
    mind = np.empty(n, dtype=np.float64)
    sse_hist = np.full(max_iter + 1, np.nan)
    shift_hist = np.full(max(max_iter, 1), np.nan)
    it = lib().oracle_lloyd(_ptr(X), n, d, k, _ptr(C), max_iter, float(tol),
                            _ptr(labels), _ptr(mind), _ptr(sse_hist),
                            _ptr(shift_hist))
    if it < 0:
        raise RuntimeError("oracle_lloyd failed: %d" % it)
    return dict(C=C, labels=labels, mind=mind, sse_hist=sse_hist[: it + 1],
                shift_hist=shift_hist[:it], iters=it)


# ---------------------------------------------------------------------------
# O4 - mixed-precision reliability test, emulated
# ---------------------------------------------------------------------------

def alpha_value(fmt: int, d: int, rho: float = 5.0, form: str = "eq") -> float:
    """Threshold alpha of the test  d^ > alpha * (||x~||^2 + ||c~||^2).

    ``form="eq"``: alpha = rho * 2 gamma^l_{d+2} (E^l of Section 4.3 with the
    test eq:quantis-reliability-test); ``form="alg"``: alpha = rho *
    gamma^l_{d+2} (the listing of alg:mp-dist); ``form="hw"``: the same
    decomposition with FP32 accumulation of exact products (a variant, not
    the paper's rule).  inf when gamma is undefined.
    """
    if form == "hw":
        # Section 4.3's two error sources re-derived for a cross term whose
        # products are exact and whose sum is accumulated in FP32:
        #   |q^ - d(x~,c~)^2| <= gamma^{32}_{d+2} (||x~||^2 + 2|x~|^T|c~| + ||c~||^2)
        #                     <= 2 gamma^{32}_{d+2} S,
        #   conversion error C <= 2(2u_l + u_l^2) (||x||^2 + ||c||^2)
        #                     <= 2(2u_l + u_l^2)(1 + u_l)^2 S,
        # with S = ||x~||^2 + ||c~||^2; the FP32 unit is taken as 2^-23.
        g32 = gamma(d + 2, 2.0 ** -23)
        if not np.isfinite(g32):
            return float("inf")
        ul = unit_roundoff(fmt)
        return rho * (2.0 * g32 + 2.0 * (2.0 * ul + ul * ul) * (1.0 + ul) ** 2)
    g = gamma(d + 2, unit_roundoff(fmt))
    if not np.isfinite(g):
        return float("inf")
    return rho * (2.0 * g if form == "eq" else g)


def mp_rows(X, C, fmt: int, alpha: float):
    """O4 for all pairs of the rows of X against C.  Returns a dict of
    (m, k) arrays: dist, q, S, A, B, cls (int8) and n_bad."""
    X, C = _f32(X), _f32(C)
    m, d = X.shape
    k = C.shape[0]
    out = {name: np.empty((m, k), dtype=np.float64)
           for name in ("dist", "q", "S", "A", "B")}
    cls = np.empty((m, k), dtype=np.int8)
    a = float(alpha) if np.isfinite(alpha) else 1e300
    nbad = lib().oracle_mp_rows(_ptr(X), m, d, _ptr(C), k, fmt, a,
                                _ptr(out["dist"]), _ptr(out["q"]),
                                _ptr(out["S"]), _ptr(out["A"]),
                                _ptr(out["B"]), _ptr(cls))
    out["cls"] = cls
    out["n_bad"] = int(nbad)
    return out


def low_sub(a: float, b: float, fmt: int) -> float:
    """O5: a - b rounded once to format fmt (0 FP16, 1 BF16, 2 FP32); a and b
    must be values of that format."""
    return lib().oracle_low_sub(float(a), float(b), int(fmt))


def low_fma(a: float, b: float, c: float, fmt: int) -> float:
    """O5: a * b + c rounded once to format fmt (operands of that format)."""
    return lib().oracle_low_fma(float(a), float(b), float(c), int(fmt))


def round_exact(hi: float, lo: float, fmt: int) -> float:
    """O5: the exact value hi + lo (|lo| <= half an FP64 ulp of hi) rounded
    once to format fmt, ties to even."""
    return lib().oracle_round_exact(float(hi), float(lo), int(fmt))


def corr_rows(X, C, high: int, fmt: int):
    """O5 for all pairs: the value a flagged pair takes under fallback
    precision ``high`` (0 FP64, 1 FP32 on the FP32 inputs, 2 the low format
    ``fmt`` on the quantised inputs), as an (m, k) float64 array."""
    X, C = _f32(X), _f32(C)
    m, d = X.shape
    k = C.shape[0]
    out = np.empty((m, k), dtype=np.float64)
    lib().oracle_corr_rows(_ptr(X), m, d, _ptr(C), k, int(high), int(fmt), _ptr(out))
    return out


def seed_pp(X, k: int, uniforms):
    """O6: indices (int64) of the k-means++ seeds drawn with ``uniforms``."""
    X = _f32(X)
    n, d = X.shape
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    assert u.shape == (k,)
    out = np.empty(k, dtype=np.int64)
    lib().oracle_seed_pp(_ptr(X), n, d, int(k), _ptr(u), _ptr(out))
    return out


def mp_scan(X, C, fmt: int, alpha: float, labels=()):
    """The per-row quantities of the parity contract over all pairs of X
    against C, streamed (nothing of size m x k is kept): O1's label ``j1``,
    ``dj1`` = its distance, ``Bj1`` = its O4 bound, ``lo`` = min over the
    other centres of (dist - B), ``d2`` = min over the other centres of
    dist, and for each array in ``labels`` the
    distance ``dlab[t]`` and bound ``Blab[t]`` at that label; ``counts`` =
    (surely corrected, ambiguous, surely kept, overflow) over all pairs.
    ``fmt`` 0 / 1 = FP16 / BF16 with threshold ``alpha`` (< 0: never
    corrected); ``fmt`` 3 = every pair by the FP64 direct formula, compared
    in FP64 (B = 2 gamma_{d+2}(u_64) dist)."""
    X, C = _f32(X), _f32(C)
    m, d = X.shape
    k = C.shape[0]
    labs = [np.ascontiguousarray(l, dtype=np.int32).ravel() for l in labels]
    for l in labs:
        if l.shape[0] != m:
            raise ValueError("label array of length %d for %d rows" % (l.shape[0], m))
    nlab = len(labs)
    lab_arr = np.concatenate(labs) if nlab else np.zeros(1, dtype=np.int32)
    out = dict(j1=np.empty(m, dtype=np.int32), dj1=np.empty(m), Bj1=np.empty(m),
               lo=np.empty(m), d2=np.empty(m), dlab=np.empty((max(nlab, 1), m)),
               Blab=np.empty((max(nlab, 1), m)), counts=np.zeros(4, dtype=np.int64))
    a = float(alpha) if np.isfinite(alpha) else 1e300
    rc = lib().oracle_mp_scan(_ptr(X), m, d, _ptr(C), k, int(fmt), a, nlab,
                              _ptr(lab_arr), _ptr(out["j1"]), _ptr(out["dj1"]),
                              _ptr(out["Bj1"]), _ptr(out["lo"]), _ptr(out["d2"]),
                              _ptr(out["dlab"]),
                              _ptr(out["Blab"]), _ptr(out["counts"]))
    if rc != 0:
        raise MemoryError("oracle_mp_scan failed")
    out["dlab"] = out["dlab"][:nlab]
    out["Blab"] = out["Blab"][:nlab]
    return out


def mp_count(X, C, fmt: int, alpha: float):
    """Counts of (surely corrected, ambiguous, surely kept, overflow) pairs."""
    X, C = _f32(X), _f32(C)
    m, d = X.shape
    k = C.shape[0]
    counts = np.zeros(4, dtype=np.int64)
    a = float(alpha) if np.isfinite(alpha) else 1e300
    lib().oracle_mp_count(_ptr(X), m, d, _ptr(C), k, fmt, a, _ptr(counts))
    return counts


def label_gate(dist, B, labels_ref):
    """Parity gate on one block of rows: point i is gated when
    min_{j != j1} (dist_ij - B_ij) > dist_{i j1} + B_{i j1}, j1 = oracle label.
    Returns a boolean array."""
    m, k = dist.shape
    rows = np.arange(m)
    lo = dist - B
    lo[rows, labels_ref] = np.inf
    hi1 = dist[rows, labels_ref] + B[rows, labels_ref]
    return lo.min(axis=1) > hi1


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(t: int) -> None:
    lib().oracle_set_num_threads(int(t))
