"""MGM preprocessing phase (Alg. 2) in natural numbering, FP64.

For each level j: point cloud X_j, operator L_j (CSR, natural numbering of the
level), its structural pattern, the colouring used by the smoother, the
interpolation P_j = I_{j+1}^j (Sec. 3), R_j = P_j^T, and for the Poisson
problem the border vector b_j (b_1 = ones, b_{j+1} = b_j P_j; Sec. 4.4).
The coarsest level keeps a dense LU with partial pivoting of L_p, or of the
bordered matrix [L_p b_p^T; b_p 0] (Sec. 4.3, Sec. 4.4).

Level numbering: level 1 keeps the caller's point order; level j+1 lists the
WSE survivors of level j in ascending level-j index.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import coarsen, colouring, discretize, galerkin, knn, transfer


@dataclass
class Level:
    xyz: np.ndarray
    L: sp.csr_matrix
    pat: sp.csr_matrix
    colour: np.ndarray | None = None
    b: np.ndarray | None = None
    P: sp.csr_matrix | None = None
    R: sp.csr_matrix | None = None
    Ppat: sp.csr_matrix | None = None
    coarse_idx: np.ndarray | None = None
    interp_idx: np.ndarray | None = None
    rows_by_colour: list = field(default_factory=list)
    patches: dict | None = None

    @property
    def N(self):
        return self.L.shape[0]

    @property
    def ncolours(self):
        return 0 if self.colour is None else int(self.colour.max()) + 1


@dataclass
class Hierarchy:
    levels: list
    problem: str
    stencils: np.ndarray
    weights: np.ndarray
    coarse_lu: tuple
    params: dict
    normals: np.ndarray | None = None


DEFAULTS = dict(disc="rbffd", phs_order=1, poly_degree=2, stencil_size=30, gfd_alpha=4.0,
                problem="screened", mu=1.0, interp_size=3, coarsen_factor=4, n_min=250,
                n_coarse_max=0, gs_block=256, gs_max_width=96)


def fine_operator(xyz, normals, params):
    """Stencils, LBO weights and L_1 (Sec. 2)."""
    sten = knn.stencils(xyz, params["stencil_size"])
    w = discretize.lbo_weights(xyz, normals, sten, params)
    L = discretize.assemble(sten, w, params["problem"], params["mu"])
    N, n = sten.shape
    pat = sp.csr_matrix((np.ones(N * n, dtype=np.int64), (np.repeat(np.arange(N), n), sten.ravel())), shape=(N, N))
    pat.sort_indices()
    return sten, w, L, pat


def build(xyz: np.ndarray, normals: np.ndarray, params: dict) -> Hierarchy:
    p = dict(DEFAULTS)
    p.update(params)
    sizes = coarsen.level_sizes(len(xyz), p["n_min"], p["n_coarse_max"], p["coarsen_factor"])
    if len(sizes) < 2:
        raise ValueError("need at least two levels")
    sten, w, L, pat = fine_operator(xyz, normals, p)
    levels = [Level(xyz=xyz, L=L, pat=pat)]
    if p["problem"] == "poisson":
        levels[0].b = np.ones(len(xyz))
    for j in range(len(sizes) - 1):
        lv = levels[j]
        cidx = coarsen.wse(lv.xyz, p["coarsen_factor"])
        assert len(cidx) == sizes[j + 1]
        cxyz = lv.xyz[cidx]
        P, iidx, _ = transfer.interpolation(lv.xyz, cxyz, p["interp_size"])
        R = transfer.restriction(P)
        Ppat = galerkin.pattern(P)
        LH, S = galerkin.galerkin(R, lv.L, P, lv.pat, Ppat)
        lv.P, lv.R, lv.Ppat, lv.coarse_idx, lv.interp_idx = P, R, Ppat, cidx, iidx
        nxt = Level(xyz=cxyz, L=LH, pat=S)
        if lv.b is not None:
            nxt.b = galerkin.coarse_border(lv.b, P)
        levels.append(nxt)
    for lv in levels[:-1]:
        lv.colour, lv.patches = colouring.smoother_colouring(lv.pat, lv.xyz, p["gs_block"], p["gs_max_width"])
        lv.rows_by_colour = [np.nonzero(lv.colour == c)[0] for c in range(lv.ncolours)]
    Lp = levels[-1].L.toarray()
    if p["problem"] == "poisson":
        b = levels[-1].b
        n = len(b)
        M = np.zeros((n + 1, n + 1))
        M[:n, :n] = Lp
        M[:n, n] = b
        M[n, :n] = b
        lu = sla.lu_factor(M)
    else:
        lu = sla.lu_factor(Lp)
    return Hierarchy(levels=levels, problem=p["problem"], stencils=sten, weights=w, coarse_lu=lu, params=p,
                     normals=normals)
