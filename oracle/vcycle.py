"""Gauss-Seidel smoothing and the MGM V(nu1,nu2)-cycle (and W/F cycles).

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

    def dinv_learned(self, j=0):
        return 1.0 / self.diag[j]

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


def learned_weights(ops, j):
    """Step weights of the learned smoother on level j, or None for Gauss-Seidel.
    `ops.learned` is either an N_1 x s array (the fine level) or a dict
    {level: N_j x s array}."""
    lw = getattr(ops, "learned", None)
    if lw is None:
        return None
    if isinstance(lw, dict):
        return lw.get(j)
    return lw if j == 0 else None


def learned_sweep(ops, u, f, j=0, lam=0.0):
    """Learned smoother on level j: for q = 1..s, u <- u + omega_q D^-1 (f - L u).
    Bordered system: the multiplier is held fixed at lam, as in the
    Gauss-Seidel smoother (the inexact-Uzawa form of Sec. 4.4), so each step
    uses the residual f - L u - b lam."""
    omega = learned_weights(ops, j)
    b = ops.border(j)
    for q in range(omega.shape[1]):
        res = f - ops.L(j, u)
        if b is not None and lam != 0.0:
            res = res - b * ops.dtype(lam)
        u += (omega[:, q] * ops.dinv_learned(j)) * res
    return u


def vcycle(ops, r, rho=None, nu1=1, nu2=1, post_reverse=False, capture=None, pre_reverse=False, cycle="V", level=0):
    """z = M r (Alg. 3 with zero initial guess). Bordered: returns (z, lambda).

    level > 0 runs the cycle of the sub-hierarchy that starts at that level
    (r and z then live on level `level`); `capture` then records that level.

    cycle = "V" (Alg. 3), "W" or "F" (the options Sec. 4.5 names): the
    coarse problem of level j is solved by one cycle of level j+1 (V), two W
    cycles, or an F cycle followed by a V cycle. The second visit continues
    from the first visit's iterate: it pre-smooths with the current
    multiplier, restricts the residual f - L e - b mu and the constraint
    residual rho - b . e, and adds the coarse correction to both e and mu.

    With `ops.learned` set (an N_1 x s array of step weights, or a dict of
    such arrays by level) those levels are smoothed by `learned_sweep` instead
    of Gauss-Seidel. `capture`, if a list, receives a copy of the start
    level's vector right after the coarse-grid correction (before
    post-smoothing)."""
    p = ops.nlevels()
    dt = ops.dtype
    bordered = rho is not None
    first = {"V": "V", "W": "W", "F": "F"}
    second = {"W": "W", "F": "V"}
    if cycle not in first:
        raise ValueError("cycle must be V, W or F")

    def visit(j, f, rho_j, e, mu, kind, zero_start):
        if j == p - 1:                       # exact: independent of the start
            ec, muc = ops.coarse_solve(f, rho_j)
            return np.asarray(ec, dtype=dt), muc
        lam = mu if (bordered and not zero_start) else 0.0
        lw = learned_weights(ops, j)
        for _ in range(nu1):
            if lw is not None:
                learned_sweep(ops, e, f, j, lam)
            else:
                gs_sweep(ops, j, e, f, lam, reverse=pre_reverse)
        res = f - ops.L(j, e)
        if bordered and lam != 0.0:
            res = res - ops.border(j) * dt(lam)
        fc = ops.R(j, res)
        rhoc = rho_j - ops.dot_border(j, e) if bordered else None
        ec, muc = visit(j + 1, fc, rhoc, np.zeros(ops.size(j + 1), dtype=dt), 0.0, first[kind], True)
        if kind != "V":
            ec, muc = visit(j + 1, fc, rhoc, ec, muc, second[kind], False)
        e += ops.P(j, ec)
        mu = (0.0 if zero_start else mu) + (muc if bordered else 0.0)
        if j == level and capture is not None:
            capture.append(np.array(e, dtype=np.float64))
        for _ in range(nu2):
            if lw is not None:
                learned_sweep(ops, e, f, j, mu if bordered else 0.0)
            else:
                gs_sweep(ops, j, e, f, mu if bordered else 0.0, reverse=post_reverse)
        return e, mu

    if not 0 <= level < p - 1:
        raise ValueError("start level must be a smoothed level")
    e0, mu0 = visit(level, np.asarray(r, dtype=dt), rho, np.zeros(ops.size(level), dtype=dt), 0.0, cycle, True)
    if bordered:
        return e0, mu0
    return e0


def make_preconditioner(ops, problem, nu1=1, nu2=1, post_reverse=False, pre_reverse=False, cycle="V"):
    """Preconditioner on FP64 vectors of length N (screened) or N+1 (bordered).
    pre_reverse / post_reverse select backward Gauss-Seidel sweeps (Sec. 4.3);
    cycle selects the V, W or F cycle."""
    if problem == "poisson":
        def M(v):
            z, lam = vcycle(ops, v[:-1], float(v[-1]), nu1, nu2, post_reverse, pre_reverse=pre_reverse, cycle=cycle)
            return np.concatenate([np.asarray(z, dtype=np.float64), [lam]])
    else:
        def M(v):
            return np.asarray(vcycle(ops, v, None, nu1, nu2, post_reverse, pre_reverse=pre_reverse, cycle=cycle),
                              dtype=np.float64)
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
