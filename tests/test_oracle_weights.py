"""Pins of the oracle's stencil weights that do not reuse its formulas.

RBF-FD (Sec. 2.2, eqs. phs_interp, rbf_fd_interp_system, rbf_fd_lap): the
weights are defined so that sum_j c_j u_j is the 2-D Laplacian, at the
stencil centre, of the PHS + polynomial interpolant of the data u_j. The test
builds that interpolant for random data (the interpolation system, not the
weight system), evaluates it around the centre and differentiates it by
finite differences extrapolated to zero step. A wrong Laplacian of the kernel
(the 3-D m(m+1) r^(m-2) instead of the 2-D m^2 r^(m-2), a wrong power) or of
the polynomials changes sum_j c_j u_j by far more than the tolerance, while
polynomial reproduction alone holds for any kernel term.

GFD (Sec. 2.3, eqs. wls_fd_approx_system, wls_fd_lap): c = W P (P^T W P)^-1
Lap(p) is the solution of min sum_j c_j^2 / w_j subject to P^T c = Lap(p).
The test recomputes w_j with scalar loops from the definition of the
Gaussian weight (tangential distances from the points' normals, no tangent
frame), builds its own tangent frame and monomials, and solves the KKT
system of that minimisation; dropping rho_j from the weight, or the weight
altogether, fails.
"""
import math

import numpy as np
import pytest

import synth
from oracle import discretize, knn


def _monomials(x, y, deg):
    """x^a y^b for every a + b <= deg, each exponent pair once (any order)."""
    return [x ** a * y ** b for d in range(deg + 1) for a in range(d + 1) for b in [d - a]]


def _monomial_laplacians(deg):
    """The Laplacian of each monomial above at the origin: 2 for x^2 and y^2."""
    out = []
    for d in range(deg + 1):
        for a in range(d + 1):
            b = d - a
            out.append(2.0 if (a, b) in ((2, 0), (0, 2)) else 0.0)
    return np.array(out)


def _scattered_stencil(rng, n, radius):
    """A projected stencil: the centre at the origin, then n - 1 points of a
    jittered disc, sorted by distance (as nearest-neighbour stencils are)."""
    pts = []
    while len(pts) < n - 1:
        p = rng.uniform(-radius, radius, 2)
        if 0.05 * radius < np.hypot(*p) <= radius:
            pts.append(p)
    pts = np.array(pts)
    pts = pts[np.argsort(np.hypot(pts[:, 0], pts[:, 1]))]
    return np.vstack([[0.0, 0.0], pts])


def _interpolant(xh, u, m, deg):
    """s(x) = sum_i a_i |x - xh_i|^m + sum_j b_j p_j(x) with s(xh_i) = u_i and
    sum_i a_i p_j(xh_i) = 0 (eqs. phs_interp, phs_interp_conditions)."""
    n = len(xh)
    A = np.array([[math.hypot(*(xh[i] - xh[k])) ** m for k in range(n)] for i in range(n)])
    P = np.array(_monomials(xh[:, 0], xh[:, 1], deg)).T
    L = P.shape[1]
    M = np.zeros((n + L, n + L))
    M[:n, :n] = A
    M[:n, n:] = P
    M[n:, :n] = P.T
    coef = np.linalg.solve(M, np.concatenate([u, np.zeros(L)]))
    a, b = coef[:n], coef[n:]

    def s(x, y):
        val = sum(a[i] * math.hypot(x - xh[i, 0], y - xh[i, 1]) ** m for i in range(n))
        return val + float(np.dot(b, _monomials(x, y, deg)))
    return s


def _fd_laplacian_at_origin(s, hs):
    """Five-point Laplacian of s at 0 for the steps hs, extrapolated to h = 0
    by a least-squares fit of L(h) = L0 + c1 h + c2 h^2 + c3 h^3 + c4 h^4 (the
    centre's kernel term is only C^(m-1) there, so odd powers appear)."""
    s0 = s(0.0, 0.0)
    vals = np.array([(s(h, 0.0) + s(-h, 0.0) + s(0.0, h) + s(0.0, -h) - 4.0 * s0) / (h * h) for h in hs])
    V = np.vander(np.asarray(hs), 5, increasing=True)
    coef, *_ = np.linalg.lstsq(V, vals, rcond=None)
    return coef[0]


@pytest.mark.parametrize("phs_order,deg,n,seed", [(1, 2, 30, 0), (2, 3, 50, 1), (1, 3, 50, 2), (3, 3, 20, 3)])
def test_rbffd_weights_apply_the_interpolants_laplacian(phs_order, deg, n, seed):
    rng = np.random.default_rng(seed)
    m = 2 * phs_order + 1
    radius = 0.3
    xh = _scattered_stencil(rng, n, radius)
    c = discretize.rbffd_weights(xh[None], phs_order, deg)[0]
    hs = radius * np.array([2e-3, 3e-3, 4e-3, 6e-3, 8e-3, 1.2e-2, 1.6e-2])
    for trial in range(3):
        u = rng.standard_normal(n)
        s = _interpolant(xh, u, m, deg)
        lap = _fd_laplacian_at_origin(s, hs)
        got = float(c @ u)
        scale = float(np.abs(c) @ np.abs(u))
        assert abs(got - lap) <= 1e-6 * scale, (trial, got, lap, scale)


def _tangential_dist2(x, nrm, i, j):
    """|xh|^2 of x_j in the tangent plane of x_i: |d|^2 - (n_i . d)^2, d = x_j - x_i."""
    nn = math.sqrt(sum(nrm[i, a] ** 2 for a in range(3)))
    d = [x[j, a] - x[i, a] for a in range(3)]
    dn = sum(d[a] * nrm[i, a] for a in range(3)) / nn
    return sum(v * v for v in d) - dn * dn


def _gaussian_weights(x, nrm, sten, i, alpha):
    """w_j = exp(-alpha |xh_i - xh_j|^2 / (rho_i^2 + rho_j^2)) over the stencil of
    x_i, rho_k the radius of the k-th projected stencil: the largest tangential
    distance from x_k to a point of its own stencil (Sec. 2.3)."""
    def rho2(k):
        return max(_tangential_dist2(x, nrm, k, q) for q in sten[k])
    r_i2 = rho2(i)
    return np.array([math.exp(-alpha * _tangential_dist2(x, nrm, i, j) / (r_i2 + rho2(j))) for j in sten[i]])


def _own_frame(nrm_i, rng):
    """An orthonormal tangent basis from a random vector (any in-plane rotation
    gives the same weights)."""
    nv = nrm_i / np.linalg.norm(nrm_i)
    v = rng.standard_normal(3)
    t1 = v - (v @ nv) * nv
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(nv, t1)
    return t1, t2


@pytest.mark.parametrize("deg,n,alpha", [(2, 25, 4.0), (2, 25, 16.0), (3, 20, 4.0)])
def test_gfd_weights_minimise_the_weighted_norm(deg, n, alpha):
    rng = np.random.default_rng(7)
    wl = synth.star_workload(1500, n_probe=20000)
    x, nrm = wl.xyz, wl.normals
    sten = knn.stencils(x, n)
    params = dict(disc="gfd", poly_degree=deg, gfd_alpha=alpha)
    c_all = discretize.lbo_weights(x, nrm, sten, params)
    for i in rng.choice(len(x), 12, replace=False):
        w = _gaussian_weights(x, nrm, sten, i, alpha)
        t1, t2 = _own_frame(nrm[i], rng)
        d = x[sten[i]] - x[i]
        P = np.array(_monomials(d @ t1, d @ t2, deg)).T
        L = P.shape[1]
        K = np.zeros((n + L, n + L))
        K[:n, :n] = np.diag(1.0 / w)
        K[:n, n:] = P
        K[n:, :n] = P.T
        sol = np.linalg.solve(K, np.concatenate([np.zeros(n), _monomial_laplacians(deg)]))
        c = sol[:n]
        assert np.max(np.abs(c_all[i] - c)) <= 1e-8 * np.max(np.abs(c)), i
