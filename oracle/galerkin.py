"""Galerkin coarse operators (Sec. 4.2, eq. galerkin; Sec. 4.4, eq. gco_saddle_point).

L_H = I_h^H L_h I_H^h with I_h^H = (I_H^h)^T. For the bordered Poisson system
the coarse border is b_H = b_h I_H^h (row) and I_h^H b_h^T (column); with the
transpose restriction these coincide, so the border stays symmetric.

The sparsity pattern of L_H is the structural product pattern of R, L_h and P
(no entry is dropped because its value happens to cancel), so integer work that
depends on it (the colouring) is independent of rounding.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def pattern(A: sp.csr_matrix) -> sp.csr_matrix:
    """0/1 integer matrix with the structural pattern of A."""
    B = sp.csr_matrix((np.ones(A.nnz, dtype=np.int64), A.indices.copy(), A.indptr.copy()), shape=A.shape)
    return B


def galerkin(R: sp.csr_matrix, L: sp.csr_matrix, P: sp.csr_matrix, Lpat: sp.csr_matrix, Ppat: sp.csr_matrix):
    """(L_H values on the structural pattern, structural pattern of L_H)."""
    Rpat = Ppat.T.tocsr()
    S = (Rpat @ Lpat @ Ppat).tocsr()
    S.sort_indices()
    S.data[:] = 1
    val = (R @ L @ P).tocsr()
    # embed the numeric product into the structural pattern (exact zeros kept)
    coo = val.tocoo()
    lookup = sp.csr_matrix((np.arange(1, S.nnz + 1), S.indices, S.indptr), shape=S.shape)
    pos = np.asarray(lookup[coo.row, coo.col]).ravel() - 1
    assert np.all(pos >= 0), "numeric product outside structural pattern"
    data = np.zeros(S.nnz)
    data[pos] = coo.data
    LH = sp.csr_matrix((data, S.indices.copy(), S.indptr.copy()), shape=S.shape)
    return LH, S


def coarse_border(b: np.ndarray, P: sp.csr_matrix) -> np.ndarray:
    """b_H = b_h I_H^h (as a vector)."""
    return P.T @ b
