"""Shift-invert eigensolves of the discrete Laplace-Beltrami operator on top of
the multilevel solver (Sec. 6.1: surface harmonics).

ARPACK's Arnoldi iteration (through scipy) finds the eigenvalues of D_h
closest to a shift sigma from repeated solves (D_h - sigma I) v = x. A handle
set up for the screened problem with mu = 1/sigma holds L_h = I - mu D_h =
-mu (D_h - sigma I), so every Arnoldi step is one device solve L_h y = x
(FGMRES + multilevel preconditioner) followed by the scaling v = -mu y. The
eigenvalues come back as sigma + 1/theta from ARPACK's Ritz values theta.
"""
from __future__ import annotations

import time

import numpy as np


def shift_invert_eigs(m, mu: float, k: int, v0: np.ndarray, rtol: float = 1e-10, restart: int = 40,
                      maxit: int = 400, arpack_tol: float = 1e-10, ncv: int | None = None, device: str = "cuda"):
    """Eigenvalues of D_h nearest sigma = 1/mu. `m` is an `Mgm` handle for the
    screened problem with this mu; `v0` the Arnoldi start vector (length N);
    `ncv` the number of Arnoldi vectors (ARPACK's default 2k+1 if None).
    Returns (eigenvalues sorted by real part, per-solve iteration counts,
    seconds spent inside the device solves, total seconds)."""
    import scipy.sparse.linalg as sla
    import torch

    if not (np.isfinite(mu) and mu != 0.0):
        raise ValueError("mu must be finite and non-zero")
    n = len(v0)
    sigma = 1.0 / mu
    iters: list[int] = []
    solve_s = [0.0]
    u = torch.zeros(n, dtype=torch.float64, device=device)

    def opinv(x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
        d_x = torch.from_numpy(x).to(device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = m.solve(d_x, u, krylov="fgmres", restart=restart, maxit=maxit, rtol=rtol)
        torch.cuda.synchronize()
        solve_s[0] += time.perf_counter() - t0
        if info["status"] != 0:
            raise RuntimeError(f"shifted solve did not converge: {info}")
        iters.append(info["iters"])
        return (-mu) * u.cpu().numpy()

    def dmat(x):  # D_h x = (x - L_h x) / mu, for ARPACK's bookkeeping only
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
        d_x = torch.from_numpy(x).to(device)
        y = m.apply(d_x)
        return (x - y.cpu().numpy()) / mu

    D = sla.LinearOperator((n, n), matvec=dmat, dtype=np.float64)
    Op = sla.LinearOperator((n, n), matvec=opinv, dtype=np.float64)
    t0 = time.perf_counter()
    ev = sla.eigs(D, k=k, sigma=sigma, OPinv=Op, which="LM", v0=np.asarray(v0, dtype=np.float64),
                  tol=arpack_tol, ncv=ncv, return_eigenvectors=False)
    total = time.perf_counter() - t0
    ev = ev[np.argsort(ev.real)]
    return ev, iters, solve_s[0], total
