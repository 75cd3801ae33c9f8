"""Multicolour ordering of each level for Gauss-Seidel smoothing.

The paper reorders every level by reverse Cuthill-McKee and runs
lexicographic GS in that order (Sec. 4.2, Sec. 4.3, Alg. 2, Alg. 3). Our
deviation, needed for a parallel smoother: colour the symmetrised structural
graph of L_j (i ~ j when L_ij or L_ji is a stored entry, i != j) so that rows
of one colour never couple, and run GS colour by colour. The result is exactly
sequential GS in any permutation that lists the colours in increasing order,
so it depends only on the colour of each row.

Colouring rules (integer-only, so two implementations agree bit for bit).
Plain multicolour ordering uses Jones-Plassmann with largest-degree-first
priorities; the patch-blocked ordering (below) uses recursive largest first
for the patch graph and DSATUR inside patches.
Jones-Plassmann: nodes are ranked by
(degree descending, h(i) ascending, i ascending) with
h(i) = splitmix64(i) >> 32 (the SplitMix64 finaliser of Steele, Lea & Flood,
2014); the first in that order has the highest priority. In every round, each
uncoloured node whose priority exceeds that of all its uncoloured neighbours
takes the smallest colour not used by any coloured neighbour.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def symmetric_graph(pat: sp.csr_matrix) -> sp.csr_matrix:
    """Symmetrised structural adjacency without the diagonal (sorted CSR)."""
    A = pat.copy().tocsr()
    A.data = np.ones_like(A.data, dtype=np.int64)
    G = (A + A.T).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    G.data[:] = 1
    return G


def priorities(G: sp.csr_matrix) -> np.ndarray:
    N = G.shape[0]
    deg = np.diff(G.indptr).astype(np.int64)
    h = (splitmix64(np.arange(N, dtype=np.uint64)) >> np.uint64(32)).astype(np.int64)
    order = np.lexsort((np.arange(N), h, -deg))
    prio = np.empty(N, dtype=np.int64)
    prio[order] = np.arange(N - 1, -1, -1)
    return prio


def jp_colouring(G: sp.csr_matrix) -> np.ndarray:
    """Colour of every node (int32) by the Jones-Plassmann rule above."""
    N = G.shape[0]
    prio = priorities(G)
    colour = np.full(N, -1, dtype=np.int64)
    indptr, nbr = G.indptr, G.indices
    row_of = np.repeat(np.arange(N), np.diff(indptr))
    while True:
        unc = colour < 0
        if not unc.any():
            break
        # max priority among uncoloured neighbours
        nb_p = np.where(unc[nbr], prio[nbr], -1)
        mx = np.full(N, -1, dtype=np.int64)
        np.maximum.at(mx, row_of, nb_p)
        sel = np.nonzero(unc & (prio > mx))[0]
        # smallest colour not used by coloured neighbours
        pos = np.full(N, -1, dtype=np.int64)
        pos[sel] = np.arange(len(sel))
        e = (pos[row_of] >= 0) & (colour[nbr] >= 0)
        ncol = int(colour.max()) + 2 if (colour >= 0).any() else 1
        used = np.zeros((len(sel), ncol + 1), dtype=bool)
        used[pos[row_of[e]], colour[nbr[e]]] = True
        colour[sel] = np.argmin(used, axis=1)
    return colour.astype(np.int32)


def colour_level(pat: sp.csr_matrix) -> np.ndarray:
    return jp_colouring(symmetric_graph(pat))


def dsatur_colouring(G: sp.csr_matrix) -> np.ndarray:
    """Brelaz's DSATUR rule (Comm. ACM 22, 1979): repeatedly take the
    uncoloured node with the most distinct colours among its coloured
    neighbours (its saturation), ties by larger degree, then smaller index, and
    give it the smallest colour none of its neighbours has. A heap with stale
    entries skipped on pop finds that node; the result is the rule's."""
    import heapq
    N = G.shape[0]
    indptr, nbr = G.indptr, G.indices
    deg = np.diff(indptr).astype(np.int64)
    colour = np.full(N, -1, dtype=np.int64)
    seen = [set() for _ in range(N)]
    heap = [(0, -int(deg[v]), v) for v in range(N)]
    heapq.heapify(heap)
    while heap:
        s, _, v = heapq.heappop(heap)
        if colour[v] >= 0 or -s != len(seen[v]):
            continue
        c = 0
        while c in seen[v]:
            c += 1
        colour[v] = c
        for u in nbr[indptr[v]:indptr[v + 1]]:
            if colour[u] < 0 and c not in seen[u]:
                seen[u].add(c)
                heapq.heappush(heap, (-len(seen[u]), -int(deg[u]), int(u)))
    return colour.astype(np.int32)


def rlf_colouring(G: sp.csr_matrix) -> np.ndarray:
    """Leighton's recursive-largest-first rule (J. Res. NBS 84, 1979): colour
    classes are filled one at a time. A class starts with the uncoloured node
    that has the most uncoloured neighbours; the uncoloured neighbours of a
    class member can no longer join the class ("excluded"). The class then
    repeatedly takes the still-eligible node with the most excluded neighbours
    (ties: fewer eligible neighbours, then smaller index) until no node is
    eligible. Neighbour counts are kept up to date as nodes change state."""
    N = G.shape[0]
    indptr, nbr = G.indptr, G.indices
    colour = np.full(N, -1, dtype=np.int64)
    uncoloured = np.ones(N, dtype=bool)
    n_unc = np.diff(indptr).astype(np.int64)  # uncoloured neighbours
    c = 0
    while uncoloured.any():
        eligible = uncoloured.copy()
        n_elig = n_unc.copy()                  # eligible neighbours
        n_excl = np.zeros(N, dtype=np.int64)   # excluded neighbours
        cand = np.nonzero(eligible)[0]
        v = int(cand[np.lexsort((cand, -n_unc[cand]))[0]])
        while True:
            colour[v] = c
            eligible[v] = False
            uncoloured[v] = False
            for u in nbr[indptr[v]:indptr[v + 1]]:
                n_elig[u] -= 1
                n_unc[u] -= 1
            for u in nbr[indptr[v]:indptr[v + 1]]:
                if eligible[u]:                 # u becomes excluded
                    eligible[u] = False
                    for x in nbr[indptr[u]:indptr[u + 1]]:
                        n_elig[x] -= 1
                        n_excl[x] += 1
            cand = np.nonzero(eligible)[0]
            if len(cand) == 0:
                break
            v = int(cand[np.lexsort((cand, n_elig[cand], -n_excl[cand]))[0]])
        c += 1
    return colour.astype(np.int32)


# ------------------------------------------------------------------ patches
def rcb_patches(xyz: np.ndarray, block: int) -> np.ndarray:
    """Patch id of every point by recursive coordinate bisection.

    A set of n > block points is sorted by (coordinate, index) along the axis
    of its largest bounding-box extent (the first such axis on ties) and cut
    after the first floor(nb/2)*block points, nb = ceil(n/block); both halves
    are cut again, the first before the second, and the sets of <= block points
    this ends in are numbered in that order. Every patch then holds exactly
    `block` points except the last one."""
    N = len(xyz)
    patch = np.empty(N, dtype=np.int64)
    nxt = 0
    stack = [np.arange(N)]
    while stack:
        idx = stack.pop()
        if len(idx) <= block:
            patch[idx] = nxt
            nxt += 1
            continue
        pts = xyz[idx]
        axis = int(np.argmax(pts.max(axis=0) - pts.min(axis=0)))
        idx = idx[np.lexsort((idx, pts[:, axis]))]
        cut = ((len(idx) + block - 1) // block // 2) * block
        stack.append(idx[cut:])
        stack.append(idx[:cut])
    return patch


def patch_colouring(pat: sp.csr_matrix, xyz: np.ndarray, block: int):
    """Patch-blocked multicolour ordering.

    Rows are cut into compact patches of `block` points by recursive
    coordinate bisection; the patch graph (patches coupled by any entry of the
    symmetrised pattern) is coloured by the recursive-largest-first rule (it
    needs fewer patch colours, i.e. launches, than DSATUR here), and the graph
    of the couplings inside patches by DSATUR. Rows with equal (patch colour, local colour)
    never couple, so GS over the composite colour pcolour * C + lcolour
    (C = number of local colours) is sequential GS in a permutation: one pass
    over the patch colours, each patch visiting its local colours in turn.
    Returns (composite colour, patch id per row, patch colour per patch,
    local colour per row).
    """
    G = symmetric_graph(pat)
    N = G.shape[0]
    patch = rcb_patches(xyz, block)
    npatch = int(patch.max()) + 1
    row_of = np.repeat(np.arange(N), np.diff(G.indptr))
    pi, pj = patch[row_of], patch[G.indices]
    cross = pi != pj
    PG = sp.csr_matrix((np.ones(int(cross.sum()), dtype=np.int64), (pi[cross], pj[cross])), shape=(npatch, npatch))
    PG.sum_duplicates()
    PG.sort_indices()
    PG.data[:] = 1
    pcol = rlf_colouring(PG)
    inner = ~cross
    GI = sp.csr_matrix((np.ones(int(inner.sum()), dtype=np.int64), (row_of[inner], G.indices[inner])), shape=(N, N))
    GI.sort_indices()
    lcol = dsatur_colouring(GI)
    C = int(lcol.max()) + 1
    comp = pcol[patch].astype(np.int64) * C + lcol
    return comp.astype(np.int64), patch, pcol, lcol


def max_row_length(pat: sp.csr_matrix) -> int:
    return int(np.diff(pat.indptr).max())


def smoother_colouring(pat: sp.csr_matrix, xyz: np.ndarray, block: int, max_width: int):
    """Colouring used by the smoother of one level: patch-blocked when
    block > 0 and every row has at most max_width entries (a parameter of the
    ordering, `gs_max_width`), else plain."""
    if block > 0 and max_row_length(pat) <= max_width:
        comp, patch, pcol, lcol = patch_colouring(pat, xyz, block)
        # relabel the composite colours densely (empty combinations dropped)
        used, dense = np.unique(comp, return_inverse=True)
        return dense.astype(np.int32), dict(patch=patch, pcolour=pcol, lcolour=lcol)
    return colour_level(pat), None


def is_valid_colouring(pat: sp.csr_matrix, colour: np.ndarray) -> bool:
    G = symmetric_graph(pat)
    row_of = np.repeat(np.arange(G.shape[0]), np.diff(G.indptr))
    return bool(np.all(colour[row_of] != colour[G.indices]))
