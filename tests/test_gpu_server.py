"""Continuous-batching server: results alone equal results in the mix
(bitwise), admission under a small memory budget, per-request errors,
polling and cancellation."""

import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
km = pytest.importorskip("paper_2407_12208_amd")

FP16 = km.Precision(km.KM_LOW_FP16, km.KM_ALPHA_PAPER_EQ, 5.0)


@pytest.fixture(scope="module")
def ctx():
    c = km.Context(0)
    yield c
    c.close()


def _req(i, n, d, k):
    X, _, _ = W.blobs(n, d, k, seed=7000 + i)
    return X, W.init_centroids(X, k, 8000 + i)


MIX = [(20000, 32, 16), (3000, 3, 8), (50000, 16, 64), (12000, 64, 200), (5000, 128, 40),
       (100000, 5, 32), (777, 16, 9)]


def _wait_all(srv, tickets, timeout_s=120):
    t0 = time.time()
    out = {}
    for t in tickets:
        rc = srv.poll(t, int(max(1, timeout_s - (time.time() - t0)) * 1000))
        out[t] = rc
    return out


def _check_against_lloyd(ctx, r, X, C0, iters):
    """Served result == kmeans_lloyd on the same input (bitwise); its first
    assignment pass matches the oracle's SSE (later passes of a free-running
    trajectory may differ on ungated near-ties)."""
    Cd = torch.from_numpy(C0).cuda()
    _, lab, _, h, _ = km.kmeans_lloyd(ctx, torch.from_numpy(X).cuda(), Cd, iters, prec=FP16,
                                      sse_hist=True)
    np.testing.assert_array_equal(r["C"], Cd.cpu().numpy())
    np.testing.assert_array_equal(r["labels"], lab.cpu().numpy())
    np.testing.assert_array_equal(r["sse_hist"], h.cpu().numpy())
    _, _, sse0 = oracle.assign(X, C0)
    assert r["sse_hist"][0] == pytest.approx(sse0, rel=1e-6)


@pytest.mark.parametrize("prec", ["fp16", "bf16_hw"])
def test_alone_equals_in_mix(ctx, prec):
    prec = FP16 if prec == "fp16" else km.Precision(km.KM_LOW_BF16, km.KM_ALPHA_HW, 5.0)
    iters = 6
    reqs = [_req(i, *s) for i, s in enumerate(MIX)]
    # each request alone
    alone = []
    for X, C0 in reqs:
        srv = km.Server(ctx, 1 << 31, max_active=8)
        t = srv.submit(X, C0, iters, prec=prec, want_mindist=True)
        assert srv.poll(t, -1) == 0
        alone.append(srv.result(t))
        srv.close()
    # all together
    srv = km.Server(ctx, 1 << 31, max_active=8)
    tickets = [srv.submit(X, C0, iters, prec=prec, want_mindist=True) for X, C0 in reqs]
    rcs = _wait_all(srv, tickets)
    assert all(rc == 0 for rc in rcs.values()), rcs
    for t, a in zip(tickets, alone):
        b = srv.result(t)
        np.testing.assert_array_equal(a["labels"], b["labels"])
        np.testing.assert_array_equal(a["C"], b["C"])
        np.testing.assert_array_equal(a["mindist"], b["mindist"])
        np.testing.assert_array_equal(a["sse_hist"], b["sse_hist"])
        assert a["stats"]["n_corrected"] == b["stats"]["n_corrected"]
        assert b["stats"]["iters"] == iters
    srv.close()


def test_served_equals_lloyd_and_oracle(ctx):
    X, C0 = _req(0, 20000, 32, 16)
    srv = km.Server(ctx, 1 << 30, max_active=4)
    t = srv.submit(X, C0, 20, prec=FP16)
    assert srv.poll(t, -1) == 0
    r = srv.result(t)
    srv.close()
    Cd = torch.from_numpy(C0).cuda()
    _, lab, _, h, _ = km.kmeans_lloyd(ctx, torch.from_numpy(X).cuda(), Cd, 20, prec=FP16, sse_hist=True)
    np.testing.assert_array_equal(r["C"], Cd.cpu().numpy())
    np.testing.assert_array_equal(r["labels"], lab.cpu().numpy())
    ref = oracle.lloyd(X, C0, 20)
    assert r["sse_hist"][-1] == pytest.approx(ref["sse_hist"][-1], rel=1e-6)


def test_admission_under_small_budget(ctx):
    # budget fits about two requests at a time: every request still finishes
    reqs = [_req(20 + i, 60000, 32, 32) for i in range(6)]
    budget = 40 << 20
    srv = km.Server(ctx, budget, max_active=16)
    tickets = [srv.submit(X, C0, 5, prec=FP16) for X, C0 in reqs]
    rcs = _wait_all(srv, tickets)
    assert all(rc == 0 for rc in rcs.values()), rcs
    for (X, C0), t in zip(reqs, tickets):
        _check_against_lloyd(ctx, srv.result(t), X, C0, 5)
    srv.close()


def test_request_larger_than_budget_is_refused(ctx):
    X, C0 = _req(40, 300000, 32, 16)  # ~40 MB of points alone
    srv = km.Server(ctx, 8 << 20, max_active=4)
    with pytest.raises(km.KMeansError) as e:
        srv.submit(X, C0, 3, prec=FP16)
    assert e.value.code == -4
    srv.close()


def test_bad_requests_fail_alone(ctx):
    good = _req(50, 8000, 16, 8)
    Xn = good[0].copy()
    Xn[17, 3] = np.nan
    Xr = good[0].copy()
    Xr[5, 1] = 1.0e5
    srv = km.Server(ctx, 1 << 30, max_active=8)
    tg = srv.submit(good[0], good[1], 4, prec=FP16)
    tn = srv.submit(Xn, good[1], 4, prec=FP16)
    tr = srv.submit(Xr, good[1], 4, prec=FP16)
    rc = _wait_all(srv, [tg, tn, tr])
    assert rc[tg] == 0 and rc[tn] == -3 and rc[tr] == -2
    _check_against_lloyd(ctx, srv.result(tg), good[0], good[1], 4)
    with pytest.raises(km.KMeansError) as e:
        srv.submit(np.ones((10, 0), np.float32), np.ones((2, 0), np.float32), 3)
    assert e.value.code == -1
    srv.close()


def test_poll_timeout_cancel_and_unknown(ctx):
    big = _req(60, 400000, 64, 256)
    small = _req(61, 2000, 8, 4)
    srv = km.Server(ctx, 1 << 31, max_active=1)
    tb = srv.submit(big[0], big[1], 100, prec=FP16)
    ts = srv.submit(small[0], small[1], 3, prec=FP16)  # waits: max_active = 1
    assert srv.poll(ts, 0) == 1  # still pending
    assert srv.cancel(ts) == 0
    assert srv.poll(ts, -1) == -7
    assert srv.poll(tb, -1) == 0
    assert srv.poll(123456, 0) == -6
    srv.close()


def test_served_request_stream_against_oracle(ctx):
    """A stream of requests shaped like the serving workload (d in
    {3, 16, 64, 128}, k in 8..512, n log-uniform, here up to 6e4 so the
    oracle stays quick), all submitted to one continuous-batching server.
    Every result against the oracle: the final SSE is the FP64 SSE of the
    returned labels against the returned centres; the final labels match
    the oracle's wherever its best centre is separated by more than the
    error bounds (O4 at the returned centres); the first pass's SSE equals
    the oracle's assignment of the initial centres up to near ties (the
    exact argmin's SSE is the least)."""
    from tests.gpu_helpers import check_assignment_scan
    reqs = W.request_stream(48, 0.0, 4242, n_range=(1_000, 60_000), iters=12)
    for r in reqs:
        r.materialize()
    srv = km.Server(ctx, 8 << 30, max_active=16)
    tickets = [srv.submit(r.X, r.C0, r.iters, prec=FP16) for r in reqs]
    rcs = _wait_all(srv, tickets)
    assert all(rc == 0 for rc in rcs.values()), rcs
    for r, t in zip(reqs, tickets):
        res = srv.result(t)
        C, lab, h = res["C"], res["labels"], res["sse_hist"]
        assert res["stats"]["iters"] == r.iters
        assert h[-1] == pytest.approx(oracle.sse_labels(r.X, C, lab), rel=1e-9)
        alpha = km.kmeans_alpha(FP16, r.d)
        scan = oracle.mp_scan(r.X, C, 0, alpha, [lab])
        check_assignment_scan(scan, 0, lab, None, h[-1], res["stats"]["n_corrected"],
                              check_sandwich=False)
        # first pass: the oracle's exact argmin has the least SSE; near ties
        # the bounds leave open may only add to it
        _, _, sse0 = oracle.assign(r.X, r.C0)
        assert sse0 * (1 - 1e-9) <= h[0] <= sse0 * (1 + 1e-4)
    srv.close()
