"""Heat-method geodesic distance with RBF-FD surface gradient and divergence.

TEST INFRASTRUCTURE ONLY: the plain CPU reference the device path is checked
against; only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg
may use it.

Sec. 6.3: the distance from a source point x* follows from three steps:
(1) heat flow u_t = Lap_M u from u_0 = delta(x*) up to a small time,
(2) the unit field eta = -grad_M u / |grad_M u|,
(3) the Poisson problem Lap_M phi = div_M eta, phi shifted to vanish at x*.
Step (1) takes backward-Euler steps (I - dt D_h) u^{k+1} = u^k and step (3)
is the bordered Poisson system; both are solved by FGMRES with the MGM
preconditioner. Gradient and divergence are RBF-FD in the tangent plane
(Sec. 2.1, as for the LBO in Sec. 2.2 but with first derivatives on the
right-hand side): for node i with tangent basis t1, t2 the weights g1, g2
reproduce d/dxh and d/dyh at the centre, and W_ij = g1_ij t1_i + g2_ij t2_i
gives grad u(x_i) = sum_j W_ij u_j and div v(x_i) = sum_j W_ij . v_j (the
divergence of a tangent field, taken in the tangent plane of x_i).

Readings (the paper leaves them open): u_0 is the unit vector of the source
node; each heat step starts FGMRES from the previous step's solution; the
direction is zero where the gradient vanishes.
"""
from __future__ import annotations

import numpy as np

from . import discretize, krylov, vcycle


def poly_gradient_at_origin(deg: int) -> np.ndarray:
    """(d/dx, d/dy) of the monomials x^a y^b at 0: 1 for x (resp. y), else 0."""
    ex = discretize.monomial_exponents(deg)
    gx = np.array([1.0 if (a, b) == (1, 0) else 0.0 for a, b in ex])
    gy = np.array([1.0 if (a, b) == (0, 1) else 0.0 for a, b in ex])
    return gx, gy


def rbffd_gradient_weights(xh: np.ndarray, phs_order: int, deg: int, chunk: int = 4096) -> np.ndarray:
    """Tangent-plane derivative weights (N x n x 2) for d/dxh and d/dyh at the
    centre: the PHS + polynomial saddle system of eq. rbf_fd_interp_system with
    the first derivatives of the basis at the centre as right-hand side. The
    derivative of |x - x_j|^m at x = 0 is -m |x_j|^(m-2) x_j (m >= 3)."""
    if phs_order < 1:
        raise ValueError("gradient weights need a PHS order k >= 1 (r^3 or smoother)")
    N, n, _ = xh.shape
    m = 2 * phs_order + 1
    L = (deg + 1) * (deg + 2) // 2
    gx, gy = poly_gradient_at_origin(deg)
    out = np.empty((N, n, 2))
    for s0 in range(0, N, chunk):
        x = xh[s0:s0 + chunk]
        s = np.sqrt((x ** 2).sum(axis=2)).max(axis=1)
        xi = x / s[:, None, None]
        r = np.sqrt(((xi[:, :, None, :] - xi[:, None, :, :]) ** 2).sum(axis=3))
        B = len(x)
        M = np.zeros((B, n + L, n + L))
        M[:, :n, :n] = r ** m
        P = discretize.poly_matrix(xi, deg)
        M[:, :n, n:] = P
        M[:, n:, :n] = np.transpose(P, (0, 2, 1))
        rc = np.sqrt((xi ** 2).sum(axis=2))
        rhs = np.zeros((B, n + L, 2))
        rhs[:, :n, 0] = -m * rc ** (m - 2) * xi[:, :, 0]
        rhs[:, :n, 1] = -m * rc ** (m - 2) * xi[:, :, 1]
        rhs[:, n:, 0] = gx
        rhs[:, n:, 1] = gy
        sol = np.linalg.solve(M, rhs)
        out[s0:s0 + chunk] = sol[:, :n, :] / s[:, None, None]
    return out


def surface_gradient_operator(xyz, normals, sten, phs_order, deg) -> np.ndarray:
    """W (N x n x 3): W_ij = g1_ij t1_i + g2_ij t2_i."""
    xh = discretize.project_stencils(xyz, normals, sten)
    g = rbffd_gradient_weights(xh, phs_order, deg)
    t1, t2 = discretize.tangent_frames(normals)
    return g[:, :, 0, None] * t1[:, None, :] + g[:, :, 1, None] * t2[:, None, :]


def gradient(W, sten, u):
    """grad_M u at every node (N x 3)."""
    return np.einsum("inc,in->ic", W, u[sten])


def divergence(W, sten, v):
    """div_M v at every node for a field v given as N x 3."""
    return np.einsum("inc,inc->i", W, v[sten])


def heat_direction(W, sten, u):
    """eta = -grad u / |grad u| (zero where the gradient vanishes)."""
    g = gradient(W, sten, u)
    nrm = np.sqrt((g * g).sum(axis=1))
    out = np.zeros_like(g)
    nz = nrm > 0
    out[nz] = -g[nz] / nrm[nz, None]
    return out


def heat_geodesic(H_heat, H_pois, W, sten, source: int, steps: int = 3, tol: float = 1e-8, restart: int = 40,
                  maxit: int = 400):
    """Steps (1)-(3) with the oracle's FGMRES + MGM. H_heat: screened
    hierarchy with mu = dt; H_pois: Poisson hierarchy of the same points.
    Returns (phi, iteration counts of the heat steps and of the Poisson solve)."""
    N = W.shape[0]
    A_h = vcycle.make_operator(H_heat)
    M_h = vcycle.make_preconditioner(vcycle.Fp64Ops(H_heat), H_heat.problem)
    u = np.zeros(N)
    u[source] = 1.0
    iters = []
    for _ in range(steps):
        u, info = krylov.fgmres(A_h, M_h, u, tol=tol, restart=restart, maxit=maxit, x0=u)
        if not info.converged:
            raise RuntimeError("heat step did not converge")
        iters.append(info.iters)
    eta = heat_direction(W, sten, u)
    rhs = np.concatenate([divergence(W, sten, eta), [0.0]])
    A_p = vcycle.make_operator(H_pois)
    M_p = vcycle.make_preconditioner(vcycle.Fp64Ops(H_pois), H_pois.problem)
    x, info = krylov.fgmres(A_p, M_p, rhs, tol=tol, restart=restart, maxit=maxit)
    if not info.converged:
        raise RuntimeError("Poisson solve did not converge")
    iters.append(info.iters)
    phi = x[:N] - x[source]
    return phi, iters
