"""Exact-arithmetic brute force for tiny inputs -- TEST INFRASTRUCTURE ONLY.

Everything here uses ``fractions.Fraction`` on the exact binary values of the
float32 inputs, so results carry no rounding at all.  These routines pin the
FP64 oracle: squared distances (eq:dist-direct), exhaustive argmin, cluster
means (eq:center), the SSE of eq:sse, and the exhaustively optimal partition
of a handful of points (the problem statement of Section 3).
"""

from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def exact(v) -> Fraction:
    return Fraction(float(v))


def sqdist(x, y) -> Fraction:
    return sum(((exact(a) - exact(b)) ** 2 for a, b in zip(x, y)), Fraction(0))


def dist_matrix(X, C):
    return [[sqdist(x, c) for c in C] for x in X]


def argmin_lowest(row):
    best = 0
    for j in range(1, len(row)):
        if row[j] < row[best]:
            best = j
    return best


def mean(points):
    m = len(points)
    d = len(points[0])
    return [sum((exact(p[l]) for p in points), Fraction(0)) / m for l in range(d)]


def sse_of(X, labels, centers):
    return sum((sqdist_exact_center(x, centers[j]) for x, j in zip(X, labels)),
               Fraction(0))


def sqdist_exact_center(x, c):
    """Squared distance of a float point to an exact (Fraction) centre."""
    return sum(((exact(a) - b) ** 2 for a, b in zip(x, c)), Fraction(0))


def optimal_partition(X, k):
    """Exhaustive search over all labelings with k non-empty clusters.
    Returns (best_sse, labels, means) with exact rationals."""
    n = len(X)
    best = None
    for lab in itertools.product(range(k), repeat=n):
        if lab[0] != 0:
            continue  # fix the label of point 0 to break symmetry
        if len(set(lab)) != k:
            continue
        means = [mean([X[i] for i in range(n) if lab[i] == j]) for j in range(k)]
        s = sse_of(X, lab, means)
        if best is None or s < best[0]:
            best = (s, list(lab), means)
    return best


def to_array(fr_list):
    return np.array([float(v) for v in fr_list])
