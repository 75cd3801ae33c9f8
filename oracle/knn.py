"""Nearest-neighbour stencils (paper Sec. 2: the n nearest points of X_h to
each centre, Euclidean distance in R^3, the centre itself included and listed
first; Sec. 3 uses the same rule for the m nearest coarse points).

Ordering key (our reading, fixed so that two implementations agree bit for
bit): (d2, index) ascending, where d2 = ((dx*dx) + (dy*dy)) + dz*dz in IEEE
double, each operation rounded separately (no fused multiply-add).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


class DuplicatePointsError(ValueError):
    pass


def sq_dist(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """d2 between rows of a and b (broadcast), in the fixed operation order."""
    dx = b[..., 0] - a[..., 0]
    dy = b[..., 1] - a[..., 1]
    dz = b[..., 2] - a[..., 2]
    return (dx * dx + dy * dy) + dz * dz


def knn(queries: np.ndarray, data: np.ndarray, k: int):
    """Indices (into `data`) and d2 of the k nearest data points of each query.

    Candidates come from a k-d tree; they are re-keyed with `sq_dist` and the
    candidate count is widened until the k-th key is provably below every
    point the tree left out.
    """
    nq, nd = len(queries), len(data)
    if k > nd:
        raise ValueError("k exceeds number of data points")
    tree = cKDTree(data)
    out_idx = np.empty((nq, k), dtype=np.int64)
    out_d2 = np.empty((nq, k))
    todo = np.arange(nq)
    kk = min(k + 8, nd)
    while len(todo):
        dist, idx = tree.query(queries[todo], kk)
        if kk == 1:
            dist, idx = dist[:, None], idx[:, None]
        d2 = sq_dist(queries[todo][:, None, :], data[idx])
        rows = np.repeat(np.arange(len(todo)), kk)
        order = np.lexsort((idx.ravel(), d2.ravel(), rows))
        idx_s = idx.ravel()[order].reshape(len(todo), kk)
        d2_s = d2.ravel()[order].reshape(len(todo), kk)
        if kk < nd:
            bound = dist[:, -1] ** 2 * (1.0 - 1e-10)
            safe = d2_s[:, k - 1] <= bound
        else:
            safe = np.ones(len(todo), dtype=bool)
        out_idx[todo[safe]] = idx_s[safe, :k]
        out_d2[todo[safe]] = d2_s[safe, :k]
        todo = todo[~safe]
        kk = min(2 * kk, nd)
    return out_idx, out_d2


def stencils(xyz: np.ndarray, n: int) -> np.ndarray:
    """Stencil index sets sigma_i (N x n), centre first; rejects duplicate points."""
    idx, d2 = knn(xyz, xyz, n)
    if n > 1 and np.any(d2[:, 1] == 0.0):
        raise DuplicatePointsError("duplicate points in the point cloud")
    assert np.all(idx[:, 0] == np.arange(len(xyz)))
    return idx
