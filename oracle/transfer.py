"""PHS interpolation and restriction between levels (Sec. 3).

Eq. interp_fd_approx: u^h_i = sum_{j in sigma_H^i} d_ij u^H_j over the m
nearest coarse points (Euclidean distance in R^3; key as in `knn`).
Eq. rbf_fd_interp: with phi(r) = r (PHS of order k = 0) plus a constant,
[A 1; 1^T 0][d; lambda] = [s; 1], A_pq = |y_p - y_q|, s_p = |x_i - y_p|,
solved in R^3 (no tangent plane). The restriction is the transpose.

Reading: because WSE gives nested clouds, a fine point that is itself a
coarse point (nearest coarse distance exactly 0) gets the injection row e_j;
the 4x4 solve would give the same row up to rounding.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .knn import knn, sq_dist


def interpolation(fine_xyz: np.ndarray, coarse_xyz: np.ndarray, m: int = 3):
    """I_H^h as CSR (N_h x N_H); also returns the (N_h x m) coarse stencils."""
    idx, d2 = knn(fine_xyz, coarse_xyz, m)
    Nh = len(fine_xyz)
    inj = d2[:, 0] == 0.0
    rows, cols, vals = [], [], []
    # injection rows
    ii = np.nonzero(inj)[0]
    rows.append(ii)
    cols.append(idx[ii, 0])
    vals.append(np.ones(len(ii)))
    # interpolation rows: (m+1) x (m+1) saddle systems, LU with partial pivoting
    jj = np.nonzero(~inj)[0]
    if len(jj):
        y = coarse_xyz[idx[jj]]                      # (B, m, 3)
        A = np.sqrt(sq_dist(y[:, :, None, :], y[:, None, :, :]))
        B = len(jj)
        M = np.zeros((B, m + 1, m + 1))
        M[:, :m, :m] = A
        M[:, :m, m] = 1.0
        M[:, m, :m] = 1.0
        rhs = np.zeros((B, m + 1))
        rhs[:, :m] = np.sqrt(d2[jj])
        rhs[:, m] = 1.0
        d = np.linalg.solve(M, rhs[..., None])[..., 0][:, :m]
        rows.append(np.repeat(jj, m))
        cols.append(idx[jj].ravel())
        vals.append(d.ravel())
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    P = sp.csr_matrix((vals, (rows, cols)), shape=(Nh, len(coarse_xyz)))
    P.sort_indices()
    return P, idx, inj


def restriction(P: sp.csr_matrix) -> sp.csr_matrix:
    """I_h^H = (I_H^h)^T."""
    R = P.T.tocsr()
    R.sort_indices()
    return R
