"""Right-preconditioned Krylov methods around the MGM cycle (Sec. 4.6; Sec. 5
uses GMRES and BiCGSTAB with MGM as a right preconditioner, and counts
BiCGSTAB iterations as preconditioner applications).

Readings (the paper does not state them): x0 = 0; the relative residual is
|f - A x|_2 / |f|_2 (on the (N+1) bordered system for Poisson); GMRES is
restarted flexible GMRES(m) (Saad 1993) with classical Gram-Schmidt applied
twice (CGS2) and Givens rotations; it stops when the Arnoldi estimate reaches
the tolerance and then confirms with the true FP64 residual, restarting when
the estimate was optimistic. BiCGSTAB is van der Vorst's method with right
preconditioning; on convergence of the recursive residual the true residual is
checked and the iteration restarted from the current iterate if needed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla


@dataclass
class SolveInfo:
    iters: int = 0                 # preconditioner applications
    converged: bool = False
    rel_res_true: float = math.nan
    history: list = field(default_factory=list)   # relative residual estimate after each application


def fgmres(A, M, f, tol=1e-10, restart=40, maxit=500, x0=None):
    n = len(f)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    fnorm = float(np.linalg.norm(f))
    info = SolveInfo()
    if fnorm == 0.0:
        info.converged, info.rel_res_true = True, 0.0
        return x, info
    while True:
        r = f - A(x)
        beta = float(np.linalg.norm(r))
        info.rel_res_true = beta / fnorm
        if beta / fnorm <= tol:
            info.converged = True
            return x, info
        if info.iters >= maxit:
            return x, info
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            info.iters += 1
            w = A(Z[j])
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0.0:
                V[j + 1] = w / hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            est = abs(g[j + 1]) / fnorm
            info.history.append(est)
            if est <= tol or info.iters >= maxit or hn == 0.0:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k])
        x = x + Z[:k].T @ y


def bicgstab(A, M, f, tol=1e-10, maxit=500, x0=None):
    n = len(f)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    fnorm = float(np.linalg.norm(f))
    info = SolveInfo()
    if fnorm == 0.0:
        info.converged, info.rel_res_true = True, 0.0
        return x, info
    while True:
        r = f - A(x)
        info.rel_res_true = float(np.linalg.norm(r)) / fnorm
        if info.rel_res_true <= tol:
            info.converged = True
            return x, info
        if info.iters >= maxit:
            return x, info
        rhat = r.copy()
        rho_old = alpha = omega = 1.0
        v = np.zeros(n)
        p = np.zeros(n)
        first = True
        while info.iters < maxit:
            rho = float(rhat @ r)
            if rho == 0.0:
                break
            if first:
                p = r.copy()
                first = False
            else:
                beta = (rho / rho_old) * (alpha / omega)
                p = r + beta * (p - omega * v)
            phat = M(p)
            info.iters += 1
            v = A(phat)
            alpha = rho / float(rhat @ v)
            s = r - alpha * v
            sn = float(np.linalg.norm(s)) / fnorm
            if sn <= tol:
                x = x + alpha * phat
                info.history.append(sn)
                break
            info.history.append(sn)
            shat = M(s)
            info.iters += 1
            t = A(shat)
            omega = float(t @ s) / float(t @ t)
            x = x + alpha * phat + omega * shat
            r = s - omega * t
            rho_old = rho
            rn = float(np.linalg.norm(r)) / fnorm
            info.history.append(rn)
            if rn <= tol or omega == 0.0:
                break
