"""Seeded synthetic inputs for the k-means assignment path.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no distances, norms, quantisation or tests).  Both the
CPU oracle and the GPU path receive the very same float32 arrays from here.

All generators use numpy ``Generator(PCG64(seed))`` so every workload is
reproducible bit for bit.  Shapes and distributions follow the paper's
experiments (Section 6): Gaussian blobs (Section 6.2.1), random and
near-duplicate 128-dimensional feature matrices (Section 6.1, Tables
tab:per_random_near and tab:dist-streess-test) and (R,G,B,x,y) pixel features
for segmentation (Section 6.2.2).  The ImageNet images of Section 6.2.2 are not
available; :func:`segmentation_instance` draws synthetic images with colour
modes, Voronoi regions and noise instead.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng",
    "blobs",
    "init_centroids",
    "gaussian_pair",
    "cancellation_pair",
    "near_duplicates",
    "collinear",
    "segmentation_instance",
    "segmentation_batch",
    "request_stream",
    "Request",
    "LLOYD_SMALL",
    "DIST_BENCH",
    "LLOYD_LARGE",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper-shaped configurations)
# ---------------------------------------------------------------------------

#: single Lloyd solve: 20,000 points, d=32, 16 blobs, 20 iterations
LLOYD_SMALL = dict(n=20_000, d=32, k=16, iters=20, seed=1001, init_seed=2001)
#: distance-kernel benchmark: 1e6 x 128 points against 4096 x 128 centroids
DIST_BENCH = dict(n=1_000_000, d=128, k=4096, seed=1002)
#: large clustering: 2e6 points, d=64, 1024 blobs, 50 iterations
LLOYD_LARGE = dict(n=2_000_000, d=64, k=1024, iters=50, seed=1003, init_seed=2003)


def blobs(n: int, d: int, k: int, seed: int, *, center_box=(-10.0, 10.0),
          std=1.0, std_range=None, shuffle=True):
    """Isotropic Gaussian blobs.

    ``k`` centres uniform in ``center_box**d``; balanced sizes (the first
    ``n % k`` blobs get one extra point).  ``std`` is a common standard
    deviation, or, if ``std_range=(lo, hi)`` is given, each blob draws its own
    standard deviation log-uniformly in that range.

    Returns ``(X, truth, centers)`` with X float32 (n, d) row-major, truth the
    generating blob of each row (int32) and the float64 centres.
    """
    g = rng(seed)
    lo, hi = center_box
    centers = g.uniform(lo, hi, size=(k, d))
    if std_range is not None:
        a, b = std_range
        stds = np.exp(g.uniform(math.log(a), math.log(b), size=k))
    else:
        stds = np.full(k, float(std))
    sizes = np.full(k, n // k, dtype=np.int64)
    sizes[: n % k] += 1
    truth = np.repeat(np.arange(k, dtype=np.int32), sizes)
    if shuffle:
        truth = truth[g.permutation(n)]
    # one draw for all points, in their final order: X = centre + std * z
    X = g.standard_normal(size=(n, d), dtype=np.float32)
    X *= stds.astype(np.float32)[truth][:, None]
    X += centers.astype(np.float32)[truth]
    return np.ascontiguousarray(X), truth, centers


def init_centroids(X: np.ndarray, k: int, seed: int) -> np.ndarray:
    """Initial centres: the first ``k`` rows of a seeded permutation of X
    (centres drawn uniformly from the data, Section 3.1)."""
    perm = rng(seed).permutation(X.shape[0])
    return np.ascontiguousarray(X[perm[:k]].astype(np.float32))


def gaussian_pair(n: int, k: int, d: int, seed: int, *, chunk_rows=1 << 17):
    """X (n, d) and C (k, d), float32, entries i.i.d. N(0,1)."""
    g = rng(seed)
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk_rows):
        e = min(n, s + chunk_rows)
        X[s:e] = g.standard_normal(size=(e - s, d), dtype=np.float32)
    C = g.standard_normal(size=(k, d), dtype=np.float32)
    return X, C


def cancellation_pair(n: int, k: int, d: int, seed: int, *, offset=1.0e3,
                      spread=1.0e-2, chunk_rows=1 << 17):
    """Cancellation-prone data: every coordinate is ``offset + spread*z``,
    z ~ N(0,1), for both X and C (all points far from the origin and close to
    each other)."""
    g = rng(seed)
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk_rows):
        e = min(n, s + chunk_rows)
        z = g.standard_normal(size=(e - s, d))
        X[s:e] = (offset + spread * z).astype(np.float32)
    z = g.standard_normal(size=(k, d))
    C = (offset + spread * z).astype(np.float32)
    return X, C


def near_duplicates(m: int, d: int, seed: int, *, fraction=1.0, eps=1.0e-4,
                    zscore=True):
    """Near-far stress construction of Section 6.1.2: P has ``m`` random rows;
    a ``fraction`` of the rows of C are ``P + eps*N(0,I)`` (near duplicates of
    the matching row of P), the rest are drawn independently.

    With ``zscore`` the random rows are standardised per feature (the paper
    z-scores its inputs, Section 6).  Returns ``(P, C, near_rows)`` where
    ``near_rows`` lists the indices i with C[i] a near duplicate of P[i].
    """
    g = rng(seed)
    P = g.standard_normal(size=(m, d))
    if zscore:
        P = (P - P.mean(axis=0)) / P.std(axis=0)
    Q = g.standard_normal(size=(m, d))
    if zscore:
        Q = (Q - Q.mean(axis=0)) / Q.std(axis=0)
    n_near = int(round(fraction * m))
    near_rows = np.sort(g.permutation(m)[:n_near])
    C = Q.copy()
    C[near_rows] = P[near_rows] + eps * g.standard_normal(size=(n_near, d))
    return (np.ascontiguousarray(P.astype(np.float32)),
            np.ascontiguousarray(C.astype(np.float32)), near_rows)


def collinear(k: int, m: int, d: int, *, offset=0.0, direction="e1"):
    """Collinear points x_i = a + i*v, i = 0..k*m-1 (no randomness).

    ``direction`` "e1" gives v = e_1; "e12" gives v = e_1 + e_2 (|v|^2 = 2).
    ``offset`` is the value of every coordinate of a.
    """
    n = k * m
    v = np.zeros(d)
    v[0] = 1.0
    if direction == "e12":
        v[1] = 1.0
    a = np.full(d, float(offset))
    i = np.arange(n, dtype=np.float64)[:, None]
    X = (a[None, :] + i * v[None, :]).astype(np.float32)
    return np.ascontiguousarray(X), v, a


def segmentation_instance(seed: int, *, H=None, W=None, hw_range=(128, 1024),
                          modes_range=(3, 12), noise=0.05, outlier_frac=0.10):
    """One synthetic segmentation-shaped instance (Section 6.2.2 features).

    An H x W image is split into Voronoi cells of M seeds placed uniformly in
    the image; each cell takes one of M colour modes (RGB uniform in [0,1]),
    pixels get N(0, noise^2) colour noise clipped to [0,1], and a fraction of
    pixels is replaced by uniform RGB.  Features are (R,G,B,x,y) with x,y
    normalised to [0,1]; each feature is then min-max normalised.
    Returns ``X`` float32 (H*W, 5) and ``(H, W, M)``.
    """
    g = rng(seed)
    if H is None:
        H = int(g.integers(hw_range[0], hw_range[1] + 1))
    if W is None:
        W = int(g.integers(hw_range[0], hw_range[1] + 1))
    M = int(g.integers(modes_range[0], modes_range[1] + 1))
    colors = g.uniform(0.0, 1.0, size=(M, 3))
    seeds = np.stack([g.uniform(0, H, size=M), g.uniform(0, W, size=M)], axis=1)
    yy = np.arange(H, dtype=np.float64)[:, None]
    xx = np.arange(W, dtype=np.float64)[None, :]
    best = np.full((H, W), np.inf)
    region = np.zeros((H, W), dtype=np.int64)
    for s in range(M):  # nearest seed, the first one on ties
        dd = (yy - seeds[s, 0]) ** 2 + (xx - seeds[s, 1]) ** 2
        region = np.where(dd < best, s, region)
        np.minimum(best, dd, out=best)
    rgb = colors[region] + noise * g.standard_normal(size=(H, W, 3))
    rgb = np.clip(rgb, 0.0, 1.0)
    out = g.uniform(0.0, 1.0, size=(H, W)) < outlier_frac
    rgb[out] = g.uniform(0.0, 1.0, size=(int(out.sum()), 3))
    feats = np.concatenate(
        [rgb.reshape(-1, 3),
         np.broadcast_to(xx / max(W - 1, 1), (H, W)).reshape(-1, 1),
         np.broadcast_to(yy / max(H - 1, 1), (H, W)).reshape(-1, 1)], axis=1)
    lo = feats.min(axis=0)
    span = feats.max(axis=0) - lo
    span[span == 0] = 1.0
    feats = (feats - lo) / span
    return np.ascontiguousarray(feats.astype(np.float32)), (H, W, M)


def segmentation_batch(count: int, seed: int, *, hw_range=(128, 1024),
                       k_range=(4, 64)):
    """``count`` independent segmentation instances with k ~ U{k_range}.

    Returns a list of dicts with keys X, k, C0 (initial centres: first k rows
    of a seeded permutation), H, W.
    """
    g = rng(seed)
    out = []
    for r in range(count):
        sub = int(g.integers(0, 2**31 - 1))
        X, (H, W, M) = segmentation_instance(sub, hw_range=hw_range)
        k = int(g.integers(k_range[0], k_range[1] + 1))
        C0 = init_centroids(X, k, sub + 1)
        out.append(dict(X=X, k=k, C0=C0, H=H, W=W, seed=sub))
    return out


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    d: int
    k: int
    seed: int
    iters: int = 30
    X: np.ndarray = field(default=None, repr=False)
    C0: np.ndarray = field(default=None, repr=False)

    def materialize(self):
        """Draw the request's blobs (k blobs, centres U[-10,10]^d, std 1)
        and its initial centres."""
        if self.X is None:
            X, _, _ = blobs(self.n, self.d, self.k, self.seed)
            self.X = X
            self.C0 = init_centroids(X, self.k, self.seed + 7)
        return self


def request_stream(count: int, rate_per_s: float, seed: int, *,
                   n_range=(1_000, 1_000_000), dims=(3, 16, 64, 128),
                   k_range=(8, 512), iters=30):
    """Poisson arrivals of k-means requests: n log-uniform in ``n_range``,
    d uniform over ``dims``, k uniform in ``k_range`` (clipped to n)."""
    g = rng(seed)
    t = 0.0
    reqs = []
    for r in range(count):
        t += float(g.exponential(1.0 / rate_per_s)) if rate_per_s > 0 else 0.0
        n = int(round(math.exp(g.uniform(math.log(n_range[0]),
                                         math.log(n_range[1])))))
        d = int(dims[int(g.integers(0, len(dims)))])
        k = int(min(g.integers(k_range[0], k_range[1] + 1), n))
        reqs.append(Request(rid=r, arrival_s=t, n=n, d=d, k=k,
                            seed=5000 + r, iters=iters))
    return reqs
