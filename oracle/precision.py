"""Reduced-precision emulation of the V-cycle (not in the paper; our reading).

FP32 mode: L_j, P_j, R_j, the border vectors and the inverse diagonal are
rounded once (round to nearest even) from their FP64 values; vectors are FP32
and every sum is an FP32 sum. FP16 row-scale mode: each row of L_j is stored
as s_i * h_ij with s_i = fp32(max_j |L_ij|) and h_ij = fp16(L_ij / s_i),
rounded once from FP64; products are formed as s_i * sum_j fp32(h_ij) x_j in
FP32; P_j and R_j stay FP32. In both modes the inverse diagonal used by GS
is 1/L~_ii of the stored operator rounded to FP32, and the coarsest solve is
the FP64 LU of the FP64 coarse operator (inputs widened, result rounded to
FP32). The outer Krylov method stays FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .vcycle import Fp64Ops


def fp16_row_scale(L: sp.csr_matrix):
    """(h as float16 CSR data, s as float32) for a CSR matrix."""
    N = L.shape[0]
    absmax = np.zeros(N)
    np.maximum.at(absmax, np.repeat(np.arange(N), np.diff(L.indptr)), np.abs(L.data))
    s = absmax.astype(np.float32)
    s = np.where(s == 0, np.float32(1.0), s)
    rows = np.repeat(np.arange(N), np.diff(L.indptr))
    h = (L.data / s.astype(np.float64)[rows]).astype(np.float16)
    return h, s


class Fp32Ops(Fp64Ops):
    dtype = np.float32

    def __init__(self, H):
        self.H = H
        self.L32 = [lv.L.astype(np.float32) for lv in H.levels]
        self.Lc = [[L[rows] for rows in lv.rows_by_colour] for L, lv in zip(self.L32, H.levels[:-1])]
        self.dinv = [(1.0 / lv.L.diagonal()).astype(np.float32) for lv in H.levels]
        self.P32 = [None if lv.P is None else lv.P.astype(np.float32) for lv in H.levels]
        self.R32 = [None if lv.R is None else lv.R.astype(np.float32) for lv in H.levels]
        self.b32 = [None if lv.b is None else lv.b.astype(np.float32) for lv in H.levels]

    def L_rows(self, j, c, u):
        return self.Lc[j][c] @ u

    def L(self, j, u):
        return self.L32[j] @ u

    def border(self, j):
        return self.b32[j]

    def gs_correction(self, j, rows, resid):
        return resid * self.dinv[j][rows]

    def dinv_learned(self, j=0):
        return self.dinv[j]

    def P(self, j, e):
        return self.P32[j] @ e

    def R(self, j, r):
        return self.R32[j] @ r

    def dot_border(self, j, e):
        return np.float32(self.b32[j] @ e)

    def coarse_solve(self, r, rho):
        r64 = np.asarray(r, dtype=np.float64)
        if rho is not None:
            x = sla.lu_solve(self.H.coarse_lu, np.concatenate([r64, [float(rho)]]))
            return x[:-1].astype(np.float32), np.float32(x[-1])
        return sla.lu_solve(self.H.coarse_lu, r64).astype(np.float32), None


class Fp16RowScaleOps(Fp32Ops):
    def __init__(self, H):
        super().__init__(H)
        self.S = []
        self.Hq = []
        self.Hc = []
        for j, lv in enumerate(H.levels):
            h, s = fp16_row_scale(lv.L)
            Hq = sp.csr_matrix((h.astype(np.float32), lv.L.indices, lv.L.indptr), shape=lv.L.shape)
            self.S.append(s)
            self.Hq.append(Hq)
            diag_q = np.asarray(Hq.diagonal(), dtype=np.float64) * s.astype(np.float64)
            self.dinv[j] = (1.0 / diag_q).astype(np.float32)
            if j < len(H.levels) - 1:
                self.Hc.append([Hq[rows] for rows in lv.rows_by_colour])

    def L_rows(self, j, c, u):
        rows = self.H.levels[j].rows_by_colour[c]
        return self.S[j][rows] * (self.Hc[j][c] @ u)

    def L(self, j, u):
        return self.S[j] * (self.Hq[j] @ u)


def ops_for(H, precision: str):
    return {"fp64": Fp64Ops, "fp32": Fp32Ops, "fp16": Fp16RowScaleOps}[precision](H)
