"""Point-cloud coarsening by weighted sample elimination, and the level count.

Sec. 4.1: the coarse cloud X_H is the subset of X_h with N_H = floor(N_h/4)
points chosen by weighted sample elimination (WSE, after Yuksel 2015), a greedy
heap-driven method that approximately maximises the Poisson-disk radius.
Alg. 2 applies it level by level, each coarse cloud taken from the previous
one. The paper gives no constants; our reading of the published method:

  * target M = floor(N / 4);
  * dbar = mean over i of the distance from x_i to its nearest other point,
    summed sequentially in index order;
  * r_max = dbar * sqrt(N / (4 M)) -- the 2-D maximal Poisson-disk radius for
    M points on an area estimated as N (sqrt(3)/2) dbar^2 (hexagonal cells);
  * neighbours: pairs with d < 2 r_max, d = sqrt(d2) (d2 as in `knn`);
  * weight w(d) = t^8, t = 1 - d/(2 r_max), formed as ((t*t)^2)^2;
  * W_i = sum of w over neighbours in ascending neighbour index;
  * repeat N - M times: remove the point of largest W (ties: smaller index)
    and subtract its weight from each remaining neighbour in ascending index;
  * survivors, in ascending index, form X_H (nested: X_H is a subset of X_h).
Yuksel's optional weight limiting is not used.

Alg. 2 line "number of levels": p = floor(log(N_1/N_min)/log 4) + 1, evaluated
here as an integer loop; alternatively coarsen while N_j > n_coarse_max.
"""
from __future__ import annotations

import heapq
import math

import numpy as np
from scipy.spatial import cKDTree

from .knn import knn, sq_dist


def wse_radius(xyz: np.ndarray, m_target: int) -> float:
    _, d2 = knn(xyz, xyz, 2)
    d = np.sqrt(d2[:, 1])
    s = 0.0
    for v in d.tolist():
        s += v
    dbar = s / len(xyz)
    return dbar * math.sqrt(len(xyz) / (4.0 * m_target))


def wse_neighbours(xyz: np.ndarray, two_r: float):
    """Sorted CSR adjacency (indptr, nbr, w) of pairs closer than two_r, with weights t^8."""
    N = len(xyz)
    tree = cKDTree(xyz)
    pairs = tree.query_pairs(two_r * (1.0 + 1e-9), output_type="ndarray")
    if len(pairs) == 0:
        pairs = np.zeros((0, 2), dtype=np.int64)
    i, j = pairs[:, 0], pairs[:, 1]
    d = np.sqrt(sq_dist(xyz[i], xyz[j]))
    keep = d < two_r
    i, j, d = i[keep], j[keep], d[keep]
    t = 1.0 - d / two_r
    t2 = t * t
    t4 = t2 * t2
    w = t4 * t4
    rows = np.concatenate([i, j])
    cols = np.concatenate([j, i])
    ws = np.concatenate([w, w])
    order = np.lexsort((cols, rows))
    rows, cols, ws = rows[order], cols[order], ws[order]
    indptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, cols, ws


def initial_weights(indptr, ws, N):
    """W_i summed in ascending neighbour order (one neighbour slot at a time)."""
    W = np.zeros(N)
    deg = np.diff(indptr)
    for slot in range(int(deg.max()) if N and len(ws) else 0):
        rows = np.nonzero(deg > slot)[0]
        W[rows] += ws[indptr[rows] + slot]
    return W


def wse(xyz: np.ndarray, factor: int = 4) -> np.ndarray:
    """Indices (ascending) of the floor(N/factor) survivors of weighted sample elimination."""
    N = len(xyz)
    M = N // factor
    r_max = wse_radius(xyz, M)
    two_r = 2.0 * r_max
    indptr, nbr, ws = wse_neighbours(xyz, two_r)
    W = initial_weights(indptr, ws, N)
    removed = np.zeros(N, dtype=bool)
    Wl = W.tolist()
    heap = [(-Wl[i], i) for i in range(N)]
    heapq.heapify(heap)
    nbr_l = nbr.tolist()
    ws_l = ws.tolist()
    ip = indptr.tolist()
    rem = removed.tolist()
    for _ in range(N - M):
        while True:
            negw, i = heapq.heappop(heap)
            if not rem[i] and -negw == Wl[i]:
                break
        rem[i] = True
        for t in range(ip[i], ip[i + 1]):
            j = nbr_l[t]
            if not rem[j]:
                Wl[j] = Wl[j] - ws_l[t]
                heapq.heappush(heap, (-Wl[j], j))
    return np.nonzero(~np.array(rem))[0]


def wse_bruteforce(xyz: np.ndarray, factor: int = 4) -> np.ndarray:
    """The same elimination by O(N^2) scanning (for pinning the heap version at tiny N)."""
    N = len(xyz)
    M = N // factor
    # nearest-other-point distances by brute force
    D2 = sq_dist(xyz[:, None, :], xyz[None, :, :])
    np.fill_diagonal(D2, np.inf)
    d = np.sqrt(D2.min(axis=1))
    s = 0.0
    for v in d.tolist():
        s += v
    r_max = (s / N) * math.sqrt(N / (4.0 * M))
    two_r = 2.0 * r_max
    D = np.sqrt(D2)
    Wm = np.zeros((N, N))
    mask = D < two_r
    t = 1.0 - D[mask] / two_r
    t2 = t * t
    t4 = t2 * t2
    Wm[mask] = t4 * t4
    W = np.zeros(N)
    for i in range(N):
        acc = 0.0
        for j in np.nonzero(mask[i])[0]:
            acc += Wm[i, j]
        W[i] = acc
    alive = np.ones(N, dtype=bool)
    for _ in range(N - M):
        Wa = np.where(alive, W, -np.inf)
        i = int(np.argmax(Wa))
        alive[i] = False
        for j in np.nonzero(mask[i] & alive)[0]:
            W[j] = W[j] - Wm[i, j]
    return np.nonzero(alive)[0]


def level_sizes(n1: int, n_min: int = 250, n_coarse_max: int = 0, factor: int = 4):
    """Level sizes N_1..N_p (Alg. 2; N_{j+1} = floor(N_j / 4)).

    With n_min > 0: p = floor(log_4(N_1/N_min)) + 1, i.e. the largest p with
    N_min * 4^(p-1) <= N_1, giving N_min <= N_p < 4 N_min. Otherwise coarsen
    while N_j > n_coarse_max.
    """
    sizes = [n1]
    if n_min > 0:
        p = 1
        while n_min * factor ** p <= n1:
            p += 1
        for _ in range(p - 1):
            sizes.append(sizes[-1] // factor)
    else:
        while sizes[-1] > n_coarse_max:
            sizes.append(sizes[-1] // factor)
    return sizes
