"""Geodesic distance by the heat method (Sec. 6.3) on top of the library.

Three steps, every one on the device: backward-Euler heat steps
(I - dt D_h) u^{k+1} = u^k from the unit vector of the source node (FGMRES +
MGM on a handle for the screened problem with mu = dt, each step started from
the previous solution), the direction eta = -grad u / |grad u| and its
divergence (the surface operators of the Poisson handle), and the bordered
Poisson solve D_h phi = div eta; phi is shifted to vanish at the source.
"""
from __future__ import annotations


def heat_distance(m_heat, m_pois, source: int, steps: int = 3, rtol: float = 1e-8, restart: int = 40,
                  maxit: int = 400):
    """Distance from node `source` (device FP64 tensor of length N) and the
    FGMRES iteration counts of the heat steps and of the Poisson solve. Both
    handles are built on the same points; `m_pois` must hold the surface
    operators (`surface_ops_setup`)."""
    import torch

    n = m_pois.n
    if m_heat.n != n:
        raise ValueError("the two handles must share the point cloud")
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    u[source] = 1.0
    iters = []
    for _ in range(steps):
        rhs = u.clone()
        u, info = m_heat.solve(rhs, u, krylov="fgmres", restart=restart, maxit=maxit, rtol=rtol, x0=True)
        if info["status"] != 0:
            raise RuntimeError(f"heat step did not converge: {info}")
        iters.append(info["iters"])
    eta = m_pois.surface_gradient(u, normalise=True)
    rhs = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    m_pois.surface_divergence(eta, out=rhs[:n])
    phi, info = m_pois.solve(rhs, krylov="fgmres", restart=restart, maxit=maxit, rtol=rtol)
    if info["status"] != 0:
        raise RuntimeError(f"Poisson solve did not converge: {info}")
    iters.append(info["iters"])
    d = phi[:n] - phi[source]
    return d, iters
