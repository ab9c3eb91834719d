"""Mixed-precision Lloyd k-means on MI355X (gfx950): thin Python binding.

Every function here marshals arguments to the C ABI of ``include/kmeans.h``
(``_build/libkmeans_mi355x.so``, built by ``build.py``) and converts status
codes to exceptions.  All arithmetic runs in the library's HIP kernels;
PyTorch only provides device memory and streams.  There is no fallback: if
the library is missing or the device is not gfx950 the calls raise.
"""

from __future__ import annotations

import ctypes as ct
import os
import threading
from dataclasses import dataclass

__all__ = [
    "KM_LOW_FP16", "KM_LOW_BF16", "KM_LOW_FP32", "KM_EXACT64",
    "KM_ALPHA_PAPER_EQ", "KM_ALPHA_PAPER_ALG", "KM_ALPHA_EXPLICIT", "KM_ALPHA_NONE", "KM_ALPHA_HW",
    "KM_HIGH_FP64", "KM_HIGH_FP32", "KM_HIGH_LOW",
    "KM_SYNC", "KMeansError", "Precision", "Stats", "Problem", "library_path", "lib",
    "Context", "kmeans_context_create", "kmeans_assign", "kmeans_assign_static",
    "kmeans_assign_flags", "kmeans_update",
    "kmeans_lloyd", "kmeans_lloyd_schedule", "kmeans_seed_pp", "kmeans_ari", "kmeans_ami",
    "kmeans_label_diff", "kmeans_solve_batch", "kmeans_pairwise", "kmeans_quantize",
    "kmeans_alpha", "kmeans_status_string", "Server", "kmeans_server_create",
    "kmeans_submit", "kmeans_poll", "kmeans_cancel", "kmeans_server_destroy",
    "kmeans_timing_enable", "kmeans_timing_read", "kmeans_tune_cache", "kmeans_tune_dump",
]

KM_LOW_FP16, KM_LOW_BF16, KM_LOW_FP32, KM_EXACT64 = 0, 1, 2, 3
KM_ALPHA_PAPER_EQ, KM_ALPHA_PAPER_ALG, KM_ALPHA_EXPLICIT, KM_ALPHA_NONE, KM_ALPHA_HW = 0, 1, 2, 3, 4
KM_HIGH_FP64, KM_HIGH_FP32, KM_HIGH_LOW = 0, 1, 2
KM_SYNC = 1
KM_LABELS_HINT = 2
KM_ROUND_LAUNCH = 4
KM_OK, KM_PENDING = 0, 1
(KM_ERR_ARG, KM_ERR_RANGE, KM_ERR_NONFINITE, KM_ERR_OOM, KM_ERR_DEVICE, KM_ERR_NOTFOUND,
 KM_ERR_CANCELLED, KM_ERR_UNSUPPORTED) = -1, -2, -3, -4, -5, -6, -7, -8
_STATUS_NAMES = {
    0: "KM_OK", 1: "KM_PENDING", -1: "KM_ERR_ARG", -2: "KM_ERR_RANGE",
    -3: "KM_ERR_NONFINITE", -4: "KM_ERR_OOM", -5: "KM_ERR_DEVICE",
    -6: "KM_ERR_NOTFOUND", -7: "KM_ERR_CANCELLED", -8: "KM_ERR_UNSUPPORTED",
}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "libkmeans_mi355x.so")
_lock = threading.Lock()
_lib = None


def library_path() -> str:
    return _LIB_PATH


class KMeansError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = int(code)
        name = _STATUS_NAMES.get(self.code, str(code))
        msg = "%s failed: %s (%s)" % (where, name, kmeans_status_string(code))
        super().__init__(msg)


class Precision(ct.Structure):
    _fields_ = [("low", ct.c_int32), ("alpha_mode", ct.c_int32),
                ("rho", ct.c_double), ("alpha", ct.c_double),
                ("high", ct.c_int32), ("reserved", ct.c_int32)]

    def __init__(self, low=KM_LOW_FP16, alpha_mode=KM_ALPHA_PAPER_EQ, rho=5.0,
                 alpha=0.0, high=0):
        super().__init__(int(low), int(alpha_mode), float(rho), float(alpha), int(high), 0)


class Stats(ct.Structure):
    _fields_ = [("n_corrected", ct.c_int64), ("n_pairs", ct.c_int64),
                ("iters", ct.c_int32), ("data_status", ct.c_int32),
                ("sse_last", ct.c_double), ("shift_last", ct.c_double),
                ("alpha_used", ct.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Problem(ct.Structure):
    _fields_ = [("X", ct.c_void_p), ("n", ct.c_int64), ("d", ct.c_int32),
                ("k", ct.c_int32), ("C_inout", ct.c_void_p),
                ("labels", ct.c_void_p), ("mindist", ct.c_void_p),
                ("sse_hist", ct.c_void_p), ("max_iter", ct.c_int32),
                ("tol", ct.c_double), ("stats", ct.POINTER(Stats))]


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(
                    "HIP library not built: %s (run paper_2407_12208_amd/build.py)"
                    % _LIB_PATH)
            L = ct.CDLL(_LIB_PATH)
            P, i32, i64, u32, dbl = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint32, ct.c_double
            PP = ct.POINTER(Precision)
            PS = ct.POINTER(Stats)
            sig = {
                "kmeans_context_create": [i32, ct.POINTER(P)],
                "kmeans_context_destroy": [P],
                "kmeans_assign": [P, P, i64, i32, P, i32, PP, P, P, P, PS, P, u32],
                "kmeans_assign_static": [P, P, i64, i32, P, i32, PP, P, P, P, PS, P, u32],
                "kmeans_assign_flags": [P, P, i64, i32, P, i32, PP, P, P, PS, P, u32],
                "kmeans_update": [P, P, i64, i32, P, i32, P, P, P, P, P, P, u32],
                "kmeans_lloyd": [P, P, i64, i32, i32, P, i32, dbl, PP, P, P, P, PS, P, u32],
                "kmeans_lloyd_schedule": [P, P, i64, i32, i32, P, i32, dbl, PP, PP, dbl, i32, P, P, P, PS,
                                          ct.POINTER(i32), P, u32],
                "kmeans_solve_batch": [P, ct.POINTER(Problem), i32, PP, P, u32],
                "kmeans_pairwise": [P, P, i64, i32, P, i32, PP, P, P, P, u32],
                "kmeans_quantize": [P, P, i64, i32, P, P, u32],
                "kmeans_alpha": [PP, i32, ct.POINTER(dbl)],
                "kmeans_server_create": [P, ct.c_size_t, i32, ct.POINTER(P)],
                "kmeans_submit": [P, ct.POINTER(Problem), PP, ct.POINTER(ct.c_uint64)],
                "kmeans_poll": [P, ct.c_uint64, i32],
                "kmeans_cancel": [P, ct.c_uint64],
                "kmeans_server_destroy": [P],
                "kmeans_timing_enable": [P, i32],
                "kmeans_timing_read": [P, ct.POINTER(ct.c_float), i32, ct.POINTER(i32)],
                "kmeans_tune_cache": [P, ct.c_char_p],
                "kmeans_seed_pp": [P, P, i64, i32, i32, ct.POINTER(dbl), P, P, P, u32],
                "kmeans_ari": [P, P, i64, ct.POINTER(dbl)],
                "kmeans_ami": [P, P, i64, ct.POINTER(dbl)],
                "kmeans_label_diff": [P, P, i64, ct.POINTER(dbl)],
            }
            for name, args in sig.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = i32
            L.kmeans_tune_dump.argtypes = [P, ct.c_char_p, ct.c_int64]
            L.kmeans_tune_dump.restype = ct.c_int64
            L.kmeans_status_string.argtypes = [i32]
            L.kmeans_status_string.restype = ct.c_char_p
            _lib = L
    return _lib


def kmeans_status_string(code) -> str:
    try:
        return lib().kmeans_status_string(int(code)).decode()
    except RuntimeError:
        return _STATUS_NAMES.get(int(code), "unknown")


def _check(code, where):
    if code != KM_OK:
        raise KMeansError(code, where)
    return code


# ---------------------------------------------------------------------------
# torch marshalling helpers
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype, name, numel=None, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError("%s is required" % name)
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    return ct.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(int(s.cuda_stream))


def _prec(p):
    if p is None:
        return None
    if isinstance(p, Precision):
        return ct.byref(p)
    if isinstance(p, dict):
        return ct.byref(Precision(**p))
    raise TypeError("precision must be a Precision or dict")


class Context:
    """Owns a ``km_context`` (device workspace, descriptor uploader)."""

    def __init__(self, device: int = 0):
        h = ct.c_void_p()
        _check(lib().kmeans_context_create(int(device), ct.byref(h)),
               "kmeans_context_create")
        self.handle = h
        self.device = int(device)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().kmeans_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def kmeans_context_create(device: int = 0) -> Context:
    return Context(device)


def kmeans_timing_enable(ctx: Context, enable: bool = True) -> None:
    _check(lib().kmeans_timing_enable(ctx.handle, 1 if enable else 0),
           "kmeans_timing_enable")


def kmeans_tune_cache(ctx: Context, path):
    """Make the context's tuning choices persistent in ``path`` (None: memory
    only)."""
    p = None if path is None else os.fsencode(path)
    _check(lib().kmeans_tune_cache(ctx.handle, p), "kmeans_tune_cache")


def kmeans_tune_dump(ctx: Context) -> str:
    """The context's tuning choices, one line per shape bucket: key, groups
    of 32 points per wave, the timed candidates in ms."""
    n = lib().kmeans_tune_dump(ctx.handle, None, 0)
    if n < 0:
        raise KMeansError(int(n), "kmeans_tune_dump")
    buf = ct.create_string_buffer(int(n) + 1)
    lib().kmeans_tune_dump(ctx.handle, buf, int(n) + 1)
    return buf.value.decode()


def kmeans_timing_read(ctx: Context, max_count: int = 4096):
    """Durations (ms) of the assignment-kernel launches recorded since
    kmeans_timing_enable, in launch order."""
    buf = (ct.c_float * max_count)()
    cnt = ct.c_int32()
    _check(lib().kmeans_timing_read(ctx.handle, buf, max_count, ct.byref(cnt)),
           "kmeans_timing_read")
    return [buf[i] for i in range(min(cnt.value, max_count))]


def kmeans_alpha(prec=None, d: int = 128) -> float:
    out = ct.c_double()
    _check(lib().kmeans_alpha(_prec(prec), int(d), ct.byref(out)), "kmeans_alpha")
    return out.value


def kmeans_assign(ctx: Context, X, C, prec=None, labels=None, mindist=None,
                  sse=None, stats=True, stream=None, sync=False, labels_hint=False,
                  static=False):
    """One assignment pass.  X (n,d) and C (k,d) are float32 device tensors.
    Returns ``(labels, mindist, sse, stats_dict_or_None)``; outputs not given
    are allocated (mindist and sse only when requested with ``True``).
    ``labels_hint=True``: ``labels`` holds an earlier assignment that seeds
    the search (same results, KM_LABELS_HINT).  ``static=True`` calls
    kmeans_assign_static (the library allocates nothing; the caller passes
    every output it wants)."""
    torch = _torch()
    n, d = X.shape
    k = C.shape[0]
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    if mindist is True:
        mindist = torch.empty(n, dtype=torch.float32, device=X.device)
    if sse is True:
        sse = torch.zeros(1, dtype=torch.float64, device=X.device)
    st = Stats() if stats else None
    fn = lib().kmeans_assign_static if static else lib().kmeans_assign
    code = fn(
        ctx.handle, _dev_ptr(X, torch.float32, "X", n * d), n, d,
        _dev_ptr(C, torch.float32, "C", k * d), k, _prec(prec),
        _dev_ptr(labels, torch.int32, "labels", n),
        _dev_ptr(mindist, torch.float32, "mindist", n, allow_none=True),
        _dev_ptr(sse, torch.float64, "sse", 1, allow_none=True),
        ct.byref(st) if st is not None else None, _stream_ptr(stream),
        (KM_SYNC if sync else 0) | (KM_LABELS_HINT if labels_hint else 0))
    _check(code, "kmeans_assign_static" if static else "kmeans_assign")
    return labels, mindist, sse, (st.as_dict() if st is not None else None)


def kmeans_assign_static(ctx: Context, X, C, prec=None, labels=None, mindist=None,
                         sse=None, stats=True, stream=None, sync=False, labels_hint=False):
    """kmeans_assign through the entry point that allocates nothing (fixed
    per-device workspace; overlapping calls on one device must be ordered
    by the caller)."""
    return kmeans_assign(ctx, X, C, prec, labels, mindist, sse, stats, stream, sync,
                         labels_hint, static=True)


def kmeans_assign_flags(ctx: Context, X, C, prec=None, labels=None, flagged=None,
                        stats=True, stream=None, sync=False, labels_hint=False):
    """The assignment pass with its per-pair fallback decisions: returns
    ``(labels, flagged (n,k) uint8, stats_dict_or_None)``."""
    torch = _torch()
    n, d = X.shape
    k = C.shape[0]
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    if flagged is None:
        flagged = torch.empty((n, k), dtype=torch.uint8, device=X.device)
    st = Stats() if stats else None
    code = lib().kmeans_assign_flags(
        ctx.handle, _dev_ptr(X, torch.float32, "X", n * d), n, d,
        _dev_ptr(C, torch.float32, "C", k * d), k, _prec(prec),
        _dev_ptr(labels, torch.int32, "labels", n),
        _dev_ptr(flagged, torch.uint8, "flagged", n * k),
        ct.byref(st) if st is not None else None, _stream_ptr(stream),
        (KM_SYNC if sync else 0) | (KM_LABELS_HINT if labels_hint else 0))
    _check(code, "kmeans_assign_flags")
    return labels, flagged, (st.as_dict() if st is not None else None)


def kmeans_pairwise(ctx: Context, X, C, prec=None, D=None, flagged=None,
                    stream=None, sync=True):
    """Materialised per-pair values (m,k) float32 and flags (m,k) uint8."""
    torch = _torch()
    m, d = X.shape
    k = C.shape[0]
    if D is None:
        D = torch.empty((m, k), dtype=torch.float32, device=X.device)
    if flagged is True:
        flagged = torch.empty((m, k), dtype=torch.uint8, device=X.device)
    code = lib().kmeans_pairwise(
        ctx.handle, _dev_ptr(X, torch.float32, "X", m * d), m, d,
        _dev_ptr(C, torch.float32, "C", k * d), k, _prec(prec),
        _dev_ptr(D, torch.float32, "D", m * k),
        _dev_ptr(flagged, torch.uint8, "flagged", m * k, allow_none=True),
        _stream_ptr(stream), KM_SYNC if sync else 0)
    _check(code, "kmeans_pairwise")
    return D, flagged


def kmeans_quantize(ctx: Context, x, low=KM_LOW_FP16, out=None, stream=None,
                    sync=True):
    torch = _torch()
    cnt = x.numel()
    if out is None:
        out = torch.empty(cnt, dtype=torch.int16, device=x.device)
    code = lib().kmeans_quantize(
        ctx.handle, _dev_ptr(x, torch.float32, "x", cnt), cnt, int(low),
        _dev_ptr(out, torch.int16, "out", cnt), _stream_ptr(stream),
        KM_SYNC if sync else 0)
    _check(code, "kmeans_quantize")
    return out


def kmeans_update(ctx: Context, X, labels, C_old, C_new=None, counts=None,
                  shift=None, sse=None, stream=None, sync=False):
    """One centre update.  ``counts``, ``shift`` and ``sse`` are optional
    device outputs (pass True to allocate).  Returns
    ``(C_new, counts, shift, sse)``."""
    torch = _torch()
    n, d = X.shape
    k = C_old.shape[0]
    if C_new is None:
        C_new = torch.empty_like(C_old)
    if counts is True:
        counts = torch.empty(k, dtype=torch.int64, device=X.device)
    if shift is True:
        shift = torch.empty(1, dtype=torch.float64, device=X.device)
    if sse is True:
        sse = torch.empty(1, dtype=torch.float64, device=X.device)
    code = lib().kmeans_update(
        ctx.handle, _dev_ptr(X, torch.float32, "X", n * d), n, d,
        _dev_ptr(labels, torch.int32, "labels", n), k,
        _dev_ptr(C_old, torch.float32, "C_old", k * d),
        _dev_ptr(C_new, torch.float32, "C_new", k * d),
        _dev_ptr(counts, torch.int64, "counts", k, allow_none=True),
        _dev_ptr(shift, torch.float64, "shift", 1, allow_none=True),
        _dev_ptr(sse, torch.float64, "sse", 1, allow_none=True),
        _stream_ptr(stream), KM_SYNC if sync else 0)
    _check(code, "kmeans_update")
    return C_new, counts, shift, sse


def kmeans_lloyd(ctx: Context, X, C_inout, max_iter: int, tol: float = 0.0,
                 prec=None, labels=None, mindist=None, sse_hist=None,
                 stats=True, stream=None, sync=False, round_launch=False):
    """Lloyd's algorithm; C_inout (k,d) float32 is updated in place.
    ``round_launch`` sets KM_ROUND_LAUNCH (all rounds of a small problem in
    one persistent launch).
    Returns ``(C_inout, labels, mindist, sse_hist, stats)``."""
    torch = _torch()
    n, d = X.shape
    k = C_inout.shape[0]
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    if mindist is True:
        mindist = torch.empty(n, dtype=torch.float32, device=X.device)
    if sse_hist is True:
        sse_hist = torch.full((max_iter + 1,), float("nan"), dtype=torch.float64,
                              device=X.device)
    st = Stats() if stats else None
    code = lib().kmeans_lloyd(
        ctx.handle, _dev_ptr(X, torch.float32, "X", n * d), n, d, k,
        _dev_ptr(C_inout, torch.float32, "C_inout", k * d), int(max_iter),
        float(tol), _prec(prec), _dev_ptr(labels, torch.int32, "labels", n),
        _dev_ptr(mindist, torch.float32, "mindist", n, allow_none=True),
        _dev_ptr(sse_hist, torch.float64, "sse_hist", max_iter + 1, allow_none=True),
        ct.byref(st) if st is not None else None, _stream_ptr(stream),
        (KM_SYNC if sync else 0) | (KM_ROUND_LAUNCH if round_launch else 0))
    _check(code, "kmeans_lloyd")
    return C_inout, labels, mindist, sse_hist, (st.as_dict() if st is not None else None)


def _agreement(fn, name, a, b):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int32).ravel()
    b = np.ascontiguousarray(b, dtype=np.int32).ravel()
    if a.shape != b.shape:
        raise ValueError("labelings of different lengths")
    out = ct.c_double()
    _check(fn(a.ctypes.data_as(ct.c_void_p), b.ctypes.data_as(ct.c_void_p), a.shape[0],
              ct.byref(out)), name)
    return out.value


def kmeans_ari(a, b) -> float:
    """Adjusted Rand index of two host labelings (numpy int arrays)."""
    return _agreement(lib().kmeans_ari, "kmeans_ari", a, b)


def kmeans_ami(a, b) -> float:
    """Adjusted mutual information (arithmetic normaliser) of two labelings."""
    return _agreement(lib().kmeans_ami, "kmeans_ami", a, b)


def kmeans_label_diff(a, b) -> float:
    """Fraction of points whose labels differ after the best one-to-one
    matching of cluster ids (the paper's segmentation Diff)."""
    return _agreement(lib().kmeans_label_diff, "kmeans_label_diff", a, b)


def kmeans_seed_pp(ctx: Context, X, k: int, uniforms, C_out=None, idx_out=None, stream=None,
                   sync=True):
    """k-means++ seeding of k rows of X (device float32 (n,d)) with the given
    uniforms (k values in [0, 1)).  Returns ``(C, idx)`` (device tensors)."""
    import numpy as np
    torch = _torch()
    n, d = X.shape
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.shape != (k,):
        raise ValueError("need %d uniforms" % k)
    if C_out is None:
        C_out = torch.empty((k, d), dtype=torch.float32, device=X.device)
    if idx_out is None:
        idx_out = torch.empty(k, dtype=torch.int32, device=X.device)
    code = lib().kmeans_seed_pp(
        ctx.handle, _dev_ptr(X, torch.float32, "X", n * d), n, d, int(k),
        u.ctypes.data_as(ct.POINTER(ct.c_double)), _dev_ptr(C_out, torch.float32, "C_out", k * d),
        _dev_ptr(idx_out, torch.int32, "idx_out", k, allow_none=True), _stream_ptr(stream),
        KM_SYNC if sync else 0)
    _check(code, "kmeans_seed_pp")
    return C_out, idx_out


def kmeans_lloyd_schedule(ctx: Context, X, C_inout, max_iter: int, early, late,
                          switch_rel: float, max_early: int, tol: float = 0.0, labels=None,
                          mindist=None, sse_hist=None, stats=True, stream=None, sync=False):
    """Lloyd's algorithm with the precision schedule of kmeans_lloyd_schedule
    (``early`` while the round's relative SSE decrease is >= ``switch_rel``,
    at most ``max_early`` rounds, then ``late``).  Returns ``(C_inout, labels,
    mindist, sse_hist, stats, switch_round)``."""
    torch = _torch()
    n, d = X.shape
    k = C_inout.shape[0]
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    if mindist is True:
        mindist = torch.empty(n, dtype=torch.float32, device=X.device)
    if sse_hist is True:
        sse_hist = torch.full((max_iter + 1,), float("nan"), dtype=torch.float64,
                              device=X.device)
    st = Stats() if stats else None
    sw = ct.c_int32(-1)
    code = lib().kmeans_lloyd_schedule(
        ctx.handle, _dev_ptr(X, torch.float32, "X", n * d), n, d, k,
        _dev_ptr(C_inout, torch.float32, "C_inout", k * d), int(max_iter), float(tol),
        _prec(early), _prec(late), float(switch_rel), int(max_early),
        _dev_ptr(labels, torch.int32, "labels", n),
        _dev_ptr(mindist, torch.float32, "mindist", n, allow_none=True),
        _dev_ptr(sse_hist, torch.float64, "sse_hist", max_iter + 1, allow_none=True),
        ct.byref(st) if st is not None else None, ct.byref(sw), _stream_ptr(stream),
        KM_SYNC if sync else 0)
    _check(code, "kmeans_lloyd_schedule")
    return (C_inout, labels, mindist, sse_hist, (st.as_dict() if st is not None else None),
            sw.value)


@dataclass
class BatchItem:
    X: object
    C: object            # updated in place
    max_iter: int
    tol: float = 0.0
    labels: object = None
    mindist: object = None
    sse_hist: object = None


def kmeans_solve_batch(ctx: Context, items, prec=None, stream=None, sync=True,
                       with_mindist=False, with_sse=True, round_launch=False):
    """Solves a list of BatchItem (device tensors) in one set of launches.
    Fills labels / mindist / sse_hist on each item; returns per-item stats."""
    torch = _torch()
    arr = (Problem * len(items))()
    stats = [Stats() for _ in items]
    for i, it in enumerate(items):
        n, d = it.X.shape
        k = it.C.shape[0]
        if it.labels is None:
            it.labels = torch.empty(n, dtype=torch.int32, device=it.X.device)
        if with_mindist and it.mindist is None:
            it.mindist = torch.empty(n, dtype=torch.float32, device=it.X.device)
        if with_sse and it.sse_hist is None:
            it.sse_hist = torch.full((it.max_iter + 1,), float("nan"),
                                     dtype=torch.float64, device=it.X.device)
        arr[i].X = _dev_ptr(it.X, torch.float32, "X", n * d)
        arr[i].n = n
        arr[i].d = d
        arr[i].k = k
        arr[i].C_inout = _dev_ptr(it.C, torch.float32, "C", k * d)
        arr[i].labels = _dev_ptr(it.labels, torch.int32, "labels", n)
        arr[i].mindist = _dev_ptr(it.mindist, torch.float32, "mindist", n, allow_none=True)
        arr[i].sse_hist = _dev_ptr(it.sse_hist, torch.float64, "sse_hist",
                                   it.max_iter + 1, allow_none=True)
        arr[i].max_iter = int(it.max_iter)
        arr[i].tol = float(it.tol)
        arr[i].stats = ct.pointer(stats[i])
    code = lib().kmeans_solve_batch(ctx.handle, arr, len(items), _prec(prec),
                                    _stream_ptr(stream),
                                    (KM_SYNC if sync else 0) | (KM_ROUND_LAUNCH if round_launch else 0))
    _check(code, "kmeans_solve_batch")
    return [s.as_dict() for s in stats]


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------

class Server:
    """Continuous-batching server; requests use HOST (numpy) buffers."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_active: int = 64):
        h = ct.c_void_p()
        _check(lib().kmeans_server_create(ctx.handle, ct.c_size_t(int(hbm_budget_bytes)),
                                          int(max_active), ct.byref(h)),
               "kmeans_server_create")
        self.handle = h
        self.ctx = ctx
        self._keep = {}

    def submit(self, X, C0, max_iter: int, tol: float = 0.0, prec=None,
               want_mindist=False, want_sse=True):
        """X (n,d) float32, C0 (k,d) float32 numpy arrays.  Returns a ticket."""
        import numpy as np
        X = np.ascontiguousarray(X, dtype=np.float32)
        C = np.ascontiguousarray(C0, dtype=np.float32).copy()
        n, d = X.shape
        k = C.shape[0]
        labels = np.empty(n, dtype=np.int32)
        mind = np.empty(n, dtype=np.float32) if want_mindist else None
        sse = np.full(max_iter + 1, np.nan) if want_sse else None
        st = Stats()
        req = Problem()
        req.X = X.ctypes.data_as(ct.c_void_p)
        req.n = n
        req.d = d
        req.k = k
        req.C_inout = C.ctypes.data_as(ct.c_void_p)
        req.labels = labels.ctypes.data_as(ct.c_void_p)
        req.mindist = mind.ctypes.data_as(ct.c_void_p) if mind is not None else None
        req.sse_hist = sse.ctypes.data_as(ct.c_void_p) if sse is not None else None
        req.max_iter = int(max_iter)
        req.tol = float(tol)
        req.stats = ct.pointer(st)
        ticket = ct.c_uint64()
        _check(lib().kmeans_submit(self.handle, ct.byref(req), _prec(prec),
                                   ct.byref(ticket)), "kmeans_submit")
        # host buffers must stay alive until completion
        self._keep[ticket.value] = dict(X=X, C=C, labels=labels, mindist=mind,
                                        sse_hist=sse, stats=st, req=req)
        return ticket.value

    def poll(self, ticket: int, timeout_ms: int = 0) -> int:
        return lib().kmeans_poll(self.handle, ct.c_uint64(ticket), int(timeout_ms))

    def result(self, ticket: int):
        r = self._keep[ticket]
        return dict(C=r["C"], labels=r["labels"], mindist=r["mindist"],
                    sse_hist=r["sse_hist"], stats=r["stats"].as_dict())

    def release(self, ticket: int):
        self._keep.pop(ticket, None)

    def cancel(self, ticket: int) -> int:
        return lib().kmeans_cancel(self.handle, ct.c_uint64(ticket))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().kmeans_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kmeans_server_create(ctx, hbm_budget_bytes, max_active=64) -> Server:
    return Server(ctx, hbm_budget_bytes, max_active)


def kmeans_submit(srv: Server, X, C0, max_iter, tol=0.0, prec=None, **kw) -> int:
    return srv.submit(X, C0, max_iter, tol, prec, **kw)


def kmeans_poll(srv: Server, ticket: int, timeout_ms: int = 0) -> int:
    return srv.poll(ticket, timeout_ms)


def kmeans_cancel(srv: Server, ticket: int) -> int:
    return srv.cancel(ticket)


def kmeans_server_destroy(srv: Server) -> None:
    srv.close()
