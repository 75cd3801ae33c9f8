"""Gauss-Seidel smoothing and the MGM V(nu1,nu2)-cycle.

Smoother (Sec. 4.3, eq. smoother): u <- u + B^{-1}(f - L u), B the lower
triangle of L in the update order (forward GS). For the bordered Poisson
system (Sec. 4.4) the multiplier lambda is held fixed:
u <- u + B^{-1}(f - L u - b lambda) (one undamped inexact-Uzawa step).
With the multicolour order (see `colouring`), one sweep updates the rows of
colour 0, then colour 1, ..., each row using the newest values of the others;
the backward sweep takes the colours in reverse.

V-cycle (Alg. 3), in preconditioner mode (initial guess zero), with the
bordered reading of Sec. 4.4 (eq. gco_saddle_point): each level carries the
defect e_j, a multiplier correction mu_j (zero on the way down) and the scalar
constraint residual rho_j; restriction passes rho unchanged after subtracting
b_j . e_j, the coarsest level solves the bordered system directly, and
interpolation passes the multiplier correction up unchanged.

The arithmetic is delegated to an operator set (`Fp64Ops` here, the reduced
precision emulations in `precision`), so that one cycle definition serves all
precisions.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class Fp64Ops:
    """Exact FP64 operators of a hierarchy."""
    dtype = np.float64

    def __init__(self, H):
        self.H = H
        self.Lc = [[lv.L[rows] for rows in lv.rows_by_colour] for lv in H.levels[:-1]]
        self.diag = [lv.L.diagonal() for lv in H.levels]

    def nlevels(self):
        return len(self.H.levels)

    def size(self, j):
        return self.H.levels[j].N

    def rows(self, j, c):
        return self.H.levels[j].rows_by_colour[c]

    def ncolours(self, j):
        return self.H.levels[j].ncolours

    def L_rows(self, j, c, u):
        return self.Lc[j][c] @ u

    def L(self, j, u):
        return self.H.levels[j].L @ u

    def border(self, j):
        return self.H.levels[j].b

    def gs_correction(self, j, rows, resid):
        return resid / self.diag[j][rows]

    learned = None

    def dinv_learned(self):
        return 1.0 / self.diag[0]

    def P(self, j, e):
        return self.H.levels[j].P @ e

    def R(self, j, r):
        return self.H.levels[j].R @ r

    def dot_border(self, j, e):
        return float(self.H.levels[j].b @ e)

    def coarse_solve(self, r, rho):
        x = sla.lu_solve(self.H.coarse_lu, np.concatenate([r, [rho]]) if rho is not None else r)
        if rho is not None:
            return x[:-1], float(x[-1])
        return x, None


def gs_sweep(ops, j, u, f, lam=0.0, reverse=False):
    """One multicolour GS sweep on level j, in place on u."""
    cs = range(ops.ncolours(j))
    if reverse:
        cs = reversed(cs)
    b = ops.border(j)
    for c in cs:
        rows = ops.rows(j, c)
        resid = f[rows] - ops.L_rows(j, c, u)
        if b is not None and lam != 0.0:
            resid = resid - b[rows] * ops.dtype(lam)
        u[rows] += ops.gs_correction(j, rows, resid)
    return u


def learned_sweep(ops, u, f):
    """Fine-level learned smoother: for q = 1..s, u <- u + omega_q D^-1 (f - L u)."""
    omega = ops.learned
    for q in range(omega.shape[1]):
        u += (omega[:, q] * ops.dinv_learned()) * (f - ops.L(0, u))
    return u


def vcycle(ops, r, rho=None, nu1=1, nu2=1, post_reverse=False, capture=None, pre_reverse=False):
    """z = M r (Alg. 3 with zero initial guess). Bordered: returns (z, lambda).

    With `ops.learned` set (an N_1 x s array of step weights) the fine level
    is smoothed by `learned_sweep` instead of Gauss-Seidel. `capture`, if a
    list, receives a copy of the fine-level vector right after the coarse-grid
    correction (before post-smoothing)."""
    p = ops.nlevels()
    dt = ops.dtype
    rhs = [None] * p
    rhos = [None] * p
    e = [None] * p
    rhs[0] = np.asarray(r, dtype=dt)
    rhos[0] = rho
    bordered = rho is not None
    for j in range(p - 1):
        e[j] = np.zeros(ops.size(j), dtype=dt)
        for _ in range(nu1):
            if j == 0 and getattr(ops, "learned", None) is not None:
                learned_sweep(ops, e[j], rhs[j])
            else:
                gs_sweep(ops, j, e[j], rhs[j], 0.0, reverse=pre_reverse)
        res = rhs[j] - ops.L(j, e[j])
        rhs[j + 1] = ops.R(j, res)
        if bordered:
            rhos[j + 1] = rhos[j] - ops.dot_border(j, e[j])
    e[p - 1], mu = ops.coarse_solve(rhs[p - 1], rhos[p - 1])
    e[p - 1] = np.asarray(e[p - 1], dtype=dt)
    for j in range(p - 2, -1, -1):
        e[j] += ops.P(j, e[j + 1])
        if j == 0 and capture is not None:
            capture.append(np.array(e[0], dtype=np.float64))
        for _ in range(nu2):
            if j == 0 and getattr(ops, "learned", None) is not None:
                learned_sweep(ops, e[j], rhs[j])
            else:
                gs_sweep(ops, j, e[j], rhs[j], mu if bordered else 0.0, reverse=post_reverse)
    if bordered:
        return e[0], mu
    return e[0]


def make_preconditioner(ops, problem, nu1=1, nu2=1, post_reverse=False, pre_reverse=False):
    """Preconditioner on FP64 vectors of length N (screened) or N+1 (bordered).
    pre_reverse / post_reverse select backward Gauss-Seidel sweeps (Sec. 4.3)."""
    if problem == "poisson":
        def M(v):
            z, lam = vcycle(ops, v[:-1], float(v[-1]), nu1, nu2, post_reverse, pre_reverse=pre_reverse)
            return np.concatenate([np.asarray(z, dtype=np.float64), [lam]])
    else:
        def M(v):
            return np.asarray(vcycle(ops, v, None, nu1, nu2, post_reverse, pre_reverse=pre_reverse), dtype=np.float64)
    return M


def make_operator(H):
    """The FP64 system operator: L_1 (screened) or the bordered [L b^T; b 0] (Poisson)."""
    L = H.levels[0].L
    if H.problem == "poisson":
        b = H.levels[0].b

        def A(v):
            u, lam = v[:-1], v[-1]
            return np.concatenate([L @ u + b * lam, [float(b @ u)]])
    else:
        def A(v):
            return L @ v
    return A
