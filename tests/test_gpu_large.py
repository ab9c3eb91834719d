"""Large synthetic clustering at full size: 2,000,000 x 64 points from 1,024
blobs, against the oracle.

* The plain FP64 direct kernel runs the 50 Lloyd rounds of the workload; its
  SSE at every pass is compared with the oracle's own free-running run
  (tests/golden/large_fp64_trajectory.txt, written by a script that calls
  only the oracle), every round's centres with the oracle's update of the
  GPU labels (O2, within one FP32 ulp), and the final assignment over all
  rows with O1.
* The mixed FP16 -> FP64 and BF16 -> FP64 (hardware-aware threshold) solves
  are checked step-locked for five rounds at full n: each round's
  assignment over every row against O4 at the GPU's current centres, each
  update against O2 of the GPU's labels.  Label differences from O1 must all
  be ungated; their number is reported.
"""

import hashlib
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import check_assignment_scan, scan_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
km = pytest.importorskip("paper_2407_12208_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "large_fp64_trajectory.txt")


@pytest.fixture(scope="module")
def ctx():
    c = km.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def large():
    cfg = W.LLOYD_LARGE
    X, _, _ = W.blobs(cfg["n"], cfg["d"], cfg["k"], cfg["seed"], center_box=(-50, 50),
                      std_range=(0.1, 2.0))
    C0 = W.init_centroids(X, cfg["k"], cfg["init_seed"])
    return X, C0, torch.from_numpy(X).cuda()


def host(t):
    return t.cpu().numpy()


def ulp_diff(a, b):
    """Distance in FP32 units in the last place (same-sign values)."""
    ia = np.asarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, dtype=np.float32).view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


def read_golden():
    sse, hashes = [], []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or line.startswith("colsum") or not line.strip():
                continue
            t, s, h = line.split()
            sse.append(float(s))
            hashes.append(h)
    return np.array(sse), hashes


def test_large_fp64_direct_trajectory(ctx, large):
    X, C0, Xd = large
    n, d = X.shape
    k = C0.shape[0]
    gold_sse, gold_hash = read_golden()
    rounds = len(gold_sse) - 1
    p64 = km.Precision(km.KM_EXACT64)
    C = torch.from_numpy(C0).cuda()
    Cn = torch.empty_like(C)
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    sse_t = torch.empty(1, dtype=torch.float64, device="cuda")
    sse, first_off, max_ulp = [], None, 0
    for t in range(rounds):
        km.kmeans_assign(ctx, Xd, C, p64, labels=lab, stats=False)
        km.kmeans_update(ctx, Xd, lab, C, C_new=Cn, sse=sse_t, sync=True)
        sse.append(float(host(sse_t)[0]))
        # O2 from the GPU's labels: the same centres to one FP32 ulp
        ref, counts, _, _ = oracle.update(X, host(lab), host(C))
        u = int(ulp_diff(host(Cn), ref).max())
        max_ulp = max(max_ulp, u)
        assert u <= 1, "round %d: centres %d ulp from O2" % (t, u)
        h = hashlib.sha256(np.ascontiguousarray(host(Cn)).tobytes()).hexdigest()
        if first_off is None and h != gold_hash[t]:
            first_off = t
        C, Cn = Cn, C
    _, mind, sse_f, st = km.kmeans_assign(ctx, Xd, C, p64, labels=lab, mindist=True, sse=True)
    sse.append(float(host(sse_f)[0]))
    sse = np.array(sse)
    rel = np.abs(sse - gold_sse) / gold_sse
    # final assignment over every row against O1 at the GPU's final centres
    Cf = host(C)
    scan = scan_rows(X, Cf, 3, None, [host(lab)])
    rep = check_assignment_scan(scan, 0, host(lab), host(mind), sse[-1], None, bound="fp64",
                                d=d, min_coverage=0.99999)
    print("FP64 direct, %d rounds: SSE rel. err. vs the oracle's own run: first %.2g, max %.2g, "
          "final %.2g; centres bitwise on the oracle's trajectory through round %s; "
          "max %d ulp from O2; final pass coverage %.7f, %d labels differ from O1"
          % (rounds, rel[0], rel.max(), rel[-1], "all" if first_off is None else first_off - 1,
             max_ulp, rep["coverage"], rep["n_diff"]))
    # the first pass starts from the same centres: same SSE to FP64 rounding
    assert rel[0] <= 1e-12
    # free-running: the final SSE within 1e-6 of the oracle's own run
    assert rel[-1] <= 1e-6


@pytest.mark.parametrize("low,mode", [(km.KM_LOW_FP16, km.KM_ALPHA_PAPER_EQ),
                                      (km.KM_LOW_BF16, km.KM_ALPHA_HW)])
def test_large_step_locked_full_rows(ctx, large, low, mode):
    X, C0, Xd = large
    n, d = X.shape
    fmt = 0 if low == km.KM_LOW_FP16 else 1
    p = km.Precision(low, mode, 5.0)
    C = torch.from_numpy(C0).cuda()
    Cn = torch.empty_like(C)
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    diffs, ungated = [], []
    for t in range(5):
        Ch = host(C)
        _, _, _, st = km.kmeans_assign(ctx, Xd, C, p, labels=lab, stats=True, labels_hint=t > 0)
        labh = host(lab)
        scan = scan_rows(X, Ch, fmt, st["alpha_used"], [labh])
        # the oracle's own gate coverage at the initial centres (first 50,000
        # rows): 0.992 for FP16, 0.959 for BF16 with the hardware-aware bound
        rep = check_assignment_scan(scan, 0, labh, None, None, st["n_corrected"],
                                    min_coverage=0.98 if fmt == 0 else 0.93)
        diffs.append(rep["n_diff"])
        ungated.append(rep["n_ungated"])
        km.kmeans_update(ctx, Xd, lab, C, C_new=Cn, sync=True)
        ref, _, _, _ = oracle.update(X, labh, Ch)
        assert int(ulp_diff(host(Cn), ref).max()) <= 1
        C, Cn = Cn, C
    print("%s step-locked, 5 rounds over %d rows: ungated points per round %s, labels "
          "differing from O1 (all ungated) %s" % ("FP16" if fmt == 0 else "BF16-hw", n,
                                                  ungated, diffs))
