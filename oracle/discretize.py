"""Tangent-plane RBF-FD and GFD discretisations of the Laplace-Beltrami operator.

Sec. 2.1 (eqs. projection1, projection2, tp_pts): the stencil of x_i is
shifted to the origin and expressed in an orthonormal tangent basis
Q = [t1 t2] of T_{x_i}M, giving 2-D points xh_j = Q^T (x_j - x_i).

Sec. 2.2 (eqs. phs_interp, rbf_fd_interp_system, rbf_fd_lap): PHS kernel
|x|^(2k+1) plus bivariate polynomials of degree l; the weights solve
[A P; P^T 0][c; lambda] = [Lap(phi); Lap(p)] evaluated at the centre.

Sec. 2.3 (eqs. wls_fd_approx_system, wls_fd_lap): weighted least squares
with Gaussian weights w_j = exp(-alpha |xh_j|^2 / (rho_i^2 + rho_j^2));
c = W P (P^T W P)^{-1} Lap(p), computed through a QR factorisation of
W^{1/2} P.

Eq. discrete_system: L_h = D_h (Poisson) or I - mu D_h (screened).

Readings: the tangent basis takes the coordinate axis least aligned with the
normal, t1 = normalise(e - (n.e) n), t2 = n x t1 (any in-plane rotation gives
the same weights up to rounding). Coordinates are scaled by the stencil
radius s_i = max_j |xh_j| before the solve and the weights divided by s_i^2
afterwards (both discretisations are scale-equivariant). rho_j is the radius
of node j's own projected stencil.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def tangent_frames(normals: np.ndarray):
    n = normals / np.linalg.norm(normals, axis=1, keepdims=True)
    ax = np.argmin(np.abs(n), axis=1)
    e = np.zeros_like(n)
    e[np.arange(len(n)), ax] = 1.0
    t1 = e - n[np.arange(len(n)), ax][:, None] * n
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(n, t1)
    return t1, t2


def project_stencils(xyz, normals, sten):
    """Tangent-plane coordinates (N x n x 2) of every stencil (eq. tp_pts)."""
    t1, t2 = tangent_frames(normals)
    d = xyz[sten] - xyz[:, None, :]
    xh = np.einsum("inc,ic->in", d, t1)
    yh = np.einsum("inc,ic->in", d, t2)
    return np.stack([xh, yh], axis=2)


def monomial_exponents(deg: int):
    """Bivariate monomials x^a y^b by total degree, then descending a."""
    return [(d - b, b) for d in range(deg + 1) for b in range(d + 1)]


def poly_matrix(xi: np.ndarray, deg: int) -> np.ndarray:
    """P_{jq} = x_j^a y_j^b for stacked 2-D points xi (..., n, 2)."""
    cols = [xi[..., 0] ** a * xi[..., 1] ** b for a, b in monomial_exponents(deg)]
    return np.stack(cols, axis=-1)


def poly_laplacian_at_origin(deg: int) -> np.ndarray:
    """Lap(x^a y^b) at 0: 2 for x^2 and y^2, 0 otherwise."""
    return np.array([2.0 if (a, b) in ((2, 0), (0, 2)) else 0.0 for a, b in monomial_exponents(deg)])


def rbffd_weights(xh: np.ndarray, phs_order: int, deg: int, chunk: int = 4096) -> np.ndarray:
    """RBF-FD LBO weights for every projected stencil (eq. rbf_fd_lap).

    The saddle-point system is solved by LU with partial pivoting (the PHS
    block has a zero diagonal, so pivoting is needed).
    """
    N, n, _ = xh.shape
    m = 2 * phs_order + 1
    L = (deg + 1) * (deg + 2) // 2
    lp = poly_laplacian_at_origin(deg)
    out = np.empty((N, n))
    for s0 in range(0, N, chunk):
        x = xh[s0:s0 + chunk]
        s = np.sqrt((x ** 2).sum(axis=2)).max(axis=1)
        xi = x / s[:, None, None]
        r = np.sqrt(((xi[:, :, None, :] - xi[:, None, :, :]) ** 2).sum(axis=3))
        A = r ** m
        P = poly_matrix(xi, deg)
        B = len(x)
        M = np.zeros((B, n + L, n + L))
        M[:, :n, :n] = A
        M[:, :n, n:] = P
        M[:, n:, :n] = np.transpose(P, (0, 2, 1))
        rhs = np.zeros((B, n + L))
        rc = np.sqrt((xi ** 2).sum(axis=2))
        rhs[:, :n] = m * m * rc ** (m - 2)
        rhs[:, n:] = lp
        sol = np.linalg.solve(M, rhs[..., None])[..., 0]
        out[s0:s0 + chunk] = sol[:, :n] / (s * s)[:, None]
    return out


def gfd_weights(xh: np.ndarray, sten: np.ndarray, deg: int, alpha: float, chunk: int = 8192) -> np.ndarray:
    """GFD (weighted least squares) LBO weights (eq. wls_fd_lap, via QR)."""
    N, n, _ = xh.shape
    r2 = (xh ** 2).sum(axis=2)
    rho = np.sqrt(r2.max(axis=1))
    lp = poly_laplacian_at_origin(deg)
    out = np.empty((N, n))
    for s0 in range(0, N, chunk):
        x = xh[s0:s0 + chunk]
        s = rho[s0:s0 + chunk]
        w = np.exp(-alpha * r2[s0:s0 + chunk] / (s[:, None] ** 2 + rho[sten[s0:s0 + chunk]] ** 2))
        xi = x / s[:, None, None]
        sw = np.sqrt(w)
        P = poly_matrix(xi, deg)
        Q, R = np.linalg.qr(sw[:, :, None] * P)
        # z = R^{-T} Lap(p);  c = W^{1/2} Q z
        z = np.linalg.solve(np.transpose(R, (0, 2, 1)), np.broadcast_to(lp, (len(x), len(lp)))[..., None])[..., 0]
        c = sw * np.einsum("bnl,bl->bn", Q, z)
        out[s0:s0 + chunk] = c / (s * s)[:, None]
    return out


def assemble(sten: np.ndarray, weights: np.ndarray, problem: str, mu: float) -> sp.csr_matrix:
    """L_h = D_h (Poisson) or I - mu D_h (screened) as CSR (eq. discrete_system)."""
    N, n = sten.shape
    rows = np.repeat(np.arange(N), n)
    D = sp.csr_matrix((weights.ravel(), (rows, sten.ravel())), shape=(N, N))
    D.sort_indices()
    if problem == "poisson":
        return D
    L = (sp.identity(N, format="csr") - mu * D).tocsr()
    L.sort_indices()
    return L


def lbo_weights(xyz, normals, sten, params):
    xh = project_stencils(xyz, normals, sten)
    if params["disc"] == "rbffd":
        return rbffd_weights(xh, params["phs_order"], params["poly_degree"])
    return gfd_weights(xh, sten, params["poly_degree"], params.get("gfd_alpha", 4.0))
