"""The persistent round launch of small problems (all Lloyd rounds in one
cooperative launch) against one launch per phase, through the C ABI: every
output bitwise equal, for the shapes, precisions and stopping rules the
launch serves, plus the oracle on one of them."""

import numpy as np
import pytest

import oracle
import workloads as W

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
BF16 = km.Precision(km.KM_LOW_BF16, km.KM_ALPHA_PAPER_EQ, 5.0)
BF16_HW = km.Precision(km.KM_LOW_BF16, km.KM_ALPHA_HW, 5.0)
FP16_UNIFORM = km.Precision(km.KM_LOW_FP16, km.KM_ALPHA_NONE, 5.0)
FP16_TO_FP32 = km.Precision(km.KM_LOW_FP16, km.KM_ALPHA_PAPER_EQ, 5.0, high=km.KM_HIGH_FP32)


def both(ctx, X, C0, T, prec, tol=0.0):
    """kmeans_lloyd twice from the same start: persistent, then per phase."""
    out = []
    Xd = dev(X)
    for persistent in (True, False):
        Cd = dev(C0)
        _, lab, mind, h, st = km.kmeans_lloyd(ctx, Xd, Cd, T, tol=tol, prec=prec, mindist=True,
                                              sse_hist=True, round_launch=persistent)
        out.append((host(Cd), host(lab), host(mind), host(h), st))
    return out


def assert_same(a, b):
    Ca, la, ma, ha, sa = a
    Cb, lb, mb, hb, sb = b
    np.testing.assert_array_equal(Ca, Cb)
    np.testing.assert_array_equal(la, lb)
    np.testing.assert_array_equal(ma, mb)
    # unused entries of the SSE history stay NaN on both sides
    np.testing.assert_array_equal(np.isnan(ha), np.isnan(hb))
    np.testing.assert_array_equal(ha[~np.isnan(ha)], hb[~np.isnan(hb)])
    for key in ("iters", "n_corrected", "n_pairs", "data_status", "sse_last", "shift_last"):
        assert sa[key] == sb[key], key


@pytest.mark.parametrize("n,d,k,prec,T", [
    (20_000, 32, 16, FP16, 20),      # the single-solve workload
    (70_001, 5, 64, BF16_HW, 7),     # segmentation-like: d = 5, largest k
    (9_999, 8, 33, FP16, 5),         # two centre blocks, ragged tail
    (4_097, 16, 40, BF16, 6),        # BF16 at the paper's threshold below the dense switch
    (30_000, 12, 20, FP16_UNIFORM, 4),
    (12_345, 24, 48, FP16_TO_FP32, 5),
    (1, 3, 1, FP16, 3),              # one point, one centre
    (5, 4, 9, FP16, 2),              # more centres than points (empty clusters)
    (200_000, 2, 7, FP16, 3),        # many chunks, few coordinates
])
def test_rounds_equal_phase_launches(ctx, n, d, k, prec, T):
    X, _, _ = W.blobs(n, d, max(1, min(k, n)), seed=n % 1000 + d)
    C0 = W.init_centroids(X, min(k, n), 7)
    if C0.shape[0] < k:  # centres past n: far away, they stay empty
        C0 = np.concatenate([C0, np.full((k - C0.shape[0], d), 1e3, np.float32)])
    print("shape", n, d, k, flush=True)
    a, b = both(ctx, X, C0, T, prec)
    assert_same(a, b)
    assert a[4]["iters"] == T


def test_rounds_run_as_one_launch(ctx):
    # the timing record has one entry per assignment launch and one for the
    # whole persistent launch: 2 entries (rounds + final pass) instead of T+1
    X, _, _ = W.blobs(20_000, 32, 16, seed=1)
    C0 = W.init_centroids(X, 16, 2)
    Xd = dev(X)
    for persistent, want in ((True, 2), (False, 11)):
        km.kmeans_timing_enable(ctx, True)
        km.kmeans_lloyd(ctx, Xd, dev(C0), 10, prec=FP16, round_launch=persistent)
        t = km.kmeans_timing_read(ctx)
        km.kmeans_timing_enable(ctx, False)
        assert len(t) == want, (persistent, t)
        print("persistent" if persistent else "phase launches", "ms:", [round(v, 4) for v in t])


def test_rounds_tolerance_stop_equal_phase_launches(ctx):
    X, _, _ = W.blobs(20_000, 32, 16, seed=1)
    C0 = W.init_centroids(X, 16, 2)
    a, b = both(ctx, X, C0, 200, FP16, tol=1e-6)
    assert_same(a, b)
    assert 1 <= a[4]["iters"] < 200 and a[4]["shift_last"] < 1e-6
    # the rounds after the stop are not run: their history slots stay NaN
    assert np.isnan(a[3][a[4]["iters"] + 1:]).all()


def test_rounds_single_round_and_repeat(ctx):
    X, _, _ = W.blobs(3_000, 10, 12, seed=5)
    C0 = W.init_centroids(X, 12, 6)
    a, b = both(ctx, X, C0, 1, FP16)
    assert_same(a, b)
    # a second identical call gives the same bits (the control words are reset)
    c, _ = both(ctx, X, C0, 1, FP16)
    assert_same(a, c)


def test_rounds_match_oracle(ctx):
    # the persistent launch against the oracle's Lloyd run: same first pass,
    # same final SSE and centres within 1 ulp (as for the per-phase path)
    cfg = W.LLOYD_SMALL
    X, _, _ = W.blobs(cfg["n"], cfg["d"], cfg["k"], cfg["seed"])
    C0 = W.init_centroids(X, cfg["k"], cfg["init_seed"])
    T = cfg["iters"]
    Cd = dev(C0)
    _, labels, mind, h, st = km.kmeans_lloyd(ctx, dev(X), Cd, T, prec=FP16, mindist=True,
                                             sse_hist=True, round_launch=True)
    ref = oracle.lloyd(X, C0, T)
    h = host(h)
    assert h[0] == pytest.approx(ref["sse_hist"][0], rel=1e-6)
    assert h[-1] == pytest.approx(ref["sse_hist"][-1], rel=1e-6)
    C = host(Cd)
    sp = np.spacing(np.maximum(np.abs(C), np.abs(ref["C"])).astype(np.float32))
    assert (np.abs(C.astype(np.float64) - ref["C"]) <= sp).all()
    assert st["iters"] == T and st["data_status"] == 0


def _batch(ctx, inst, prec, round_launch):
    items = [km.BatchItem(X=dev(X), C=dev(C0), max_iter=T, tol=tol) for X, C0, T, tol in inst]
    stats = km.kmeans_solve_batch(ctx, items, prec, with_mindist=True, round_launch=round_launch)
    return [(host(it.C), host(it.labels), host(it.mindist), host(it.sse_hist), st)
            for it, st in zip(items, stats)]


@pytest.mark.parametrize("prec", [FP16, BF16_HW])
def test_batch_round_launch_equals_phase_launches(ctx, prec):
    # uneven problems: segmentation-shaped (d = 5, several k), blobs at d = 8,
    # 16 and 32 (three kernel shapes, so several persistent launches), a
    # tolerance stop, different round counts, and a d = 64 problem that the
    # persistent launch does not serve (it keeps its per-phase rounds)
    inst = []
    for r in range(3):
        X, _ = W.segmentation_instance(900 + r, hw_range=(64, 160))
        inst.append((X, W.init_centroids(X, 4 + 19 * r, 910 + r), 5 + r, 0.0))
    for i, (n, d, k) in enumerate([(7_001, 8, 33), (4_096, 16, 64), (20_000, 32, 16), (3_000, 64, 20)]):
        X, _, _ = W.blobs(n, d, k, seed=920 + i)
        inst.append((X, W.init_centroids(X, k, 930 + i), 6, 1e-4 if i == 2 else 0.0))
    a = _batch(ctx, inst, prec, True)
    b = _batch(ctx, inst, prec, False)
    for i, (x, y) in enumerate(zip(a, b)):
        print("problem", i, "iters", x[4]["iters"], flush=True)
        assert_same(x, y)


def test_round_launch_gives_up_a_wait_and_reports_it(ctx, monkeypatch):
    # a host-set cap of one poll per grid-wide wait forces the give-up path:
    # the waiting workgroup raises the abort flag, every workgroup leaves, the
    # launch ends and the call reports a device error; the context stays usable
    X, _, _ = W.blobs(20_000, 32, 16, seed=1)
    C0 = W.init_centroids(X, 16, 2)
    Xd = dev(X)
    monkeypatch.setenv("KM_ROUND_SPIN_LIMIT", "1")
    for tol in (0.0, 1e-6):
        with pytest.raises(km.KMeansError) as err:
            km.kmeans_lloyd(ctx, Xd, dev(C0), 20, tol=tol, prec=FP16, stats=True, round_launch=True)
        assert err.value.code == km.KM_ERR_DEVICE, err.value
    monkeypatch.delenv("KM_ROUND_SPIN_LIMIT")
    a, b = both(ctx, X, C0, 5, FP16)
    assert_same(a, b)
