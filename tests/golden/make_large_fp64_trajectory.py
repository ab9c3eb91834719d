#!/usr/bin/env python3
"""Writes large_fp64_trajectory.txt: the CPU oracle's own Lloyd run (O3,
FP64 direct formula, exact argmin, FP64 centre sums rounded once to FP32) on
the large synthetic clustering -- 2,000,000 points in 64 dimensions from
1,024 Gaussian blobs (centres U[-50,50]^64, per-blob std log-uniform in
[0.1, 2]), initial centres the first 1,024 rows of a seeded permutation, 50
rounds plus the final assignment.

Calls only ``oracle`` and ``workloads`` (seeded inputs).  Stored: the SSE of
every assignment pass and, per round, the SHA-256 of the float32 centres
after the update (so a GPU run can tell where it first leaves the oracle's
trajectory), and the final centres' coordinate sums.
Run: python tests/golden/make_large_fp64_trajectory.py  (about 15 min on 8
host threads).
"""

import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "large_fp64_trajectory.txt")


def main():
    cfg = W.LLOYD_LARGE
    X, _, _ = W.blobs(cfg["n"], cfg["d"], cfg["k"], cfg["seed"], center_box=(-50, 50),
                      std_range=(0.1, 2.0))
    C = W.init_centroids(X, cfg["k"], cfg["init_seed"])
    rounds = cfg["iters"]
    lines = ["# CPU oracle Lloyd trajectory (O3, FP64 direct), large synthetic clustering",
             "# n=%d d=%d k=%d seed=%d init_seed=%d rounds=%d" % (
                 cfg["n"], cfg["d"], cfg["k"], cfg["seed"], cfg["init_seed"], rounds),
             "# written by tests/golden/make_large_fp64_trajectory.py",
             "# columns: pass  sse_of_that_assignment  sha256_of_centres_after_update"]
    t0 = time.time()
    for t in range(rounds + 1):
        labels, _, sse = oracle.assign(X, C)
        if t < rounds:
            C, _, _, _ = oracle.update(X, labels, C)
            h = hashlib.sha256(np.ascontiguousarray(C, dtype=np.float32).tobytes()).hexdigest()
        else:
            h = "-"
        lines.append("%d %.17g %s" % (t, sse, h))
        print("pass %d sse %.17g (%.0f s)" % (t, sse, time.time() - t0), flush=True)
    sums = np.asarray(C, dtype=np.float64).sum(axis=0)
    lines.append("# final centres: sum over centres of each coordinate (FP64)")
    lines.append("colsum " + " ".join("%.17g" % v for v in sums))
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
