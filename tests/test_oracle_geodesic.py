"""Pins of the oracle's surface gradient, divergence and heat-method distance.

- The tangent-plane derivative weights reproduce d/dxh and d/dyh of every
  monomial of degree <= l at the centre (the defining conditions).
- On the unit sphere grad_M z = e_z - z n and Lap_M z = div_M grad_M z = -2z
  (z is a degree-1 spherical harmonic), to the discretisation error.
- The heat-method distance approaches the great-circle distance arccos(x.x*).
"""
import numpy as np
import pytest

import synth
from oracle import discretize, geodesic, hierarchy, knn


@pytest.fixture(scope="module")
def sphere():
    rp, _, _ = synth.rng_streams(8)
    x = synth.jittered_fibonacci_sphere(4096, rp, 0.1)
    sten = knn.stencils(x, 12)
    return x, sten, geodesic.surface_gradient_operator(x, x, sten, 2, 2)


@pytest.mark.parametrize("k,deg,n", [(2, 2, 12), (3, 3, 20), (1, 2, 9)])
def test_gradient_weights_reproduce_monomial_derivatives(sphere, k, deg, n):
    x = sphere[0]
    sten = knn.stencils(x, n)
    xh = discretize.project_stencils(x, x, sten)
    g = geodesic.rbffd_gradient_weights(xh, k, deg)
    s = np.sqrt((xh ** 2).sum(axis=2)).max(axis=1)
    for a, b in discretize.monomial_exponents(deg):
        p = xh[..., 0] ** a * xh[..., 1] ** b
        for c, exact in ((0, float((a, b) == (1, 0))), (1, float((a, b) == (0, 1)))):
            val = (g[..., c] * p).sum(axis=1)
            scale = np.abs(g[..., c]).sum(axis=1) * s ** (a + b)
            assert np.max(np.abs(val - exact) / scale) < 1e-10, (a, b, c)


def test_sphere_gradient_and_divergence(sphere):
    x, sten, W = sphere
    z = x[:, 2]
    exact = np.array([0.0, 0.0, 1.0])[None, :] - z[:, None] * x
    g = geodesic.gradient(W, sten, z)
    assert np.max(np.abs(g - exact)) < 1e-4
    assert np.max(np.abs((g * x).sum(axis=1))) < 1e-12        # tangent by construction
    assert np.max(np.abs(geodesic.divergence(W, sten, exact) + 2.0 * z)) < 3e-3
    assert np.max(np.abs(geodesic.divergence(W, sten, g) + 2.0 * z)) < 3e-3
    # a field along the normal has no tangential divergence in this discretisation
    assert np.max(np.abs(geodesic.divergence(W, sten, x * 0.0))) == 0.0


def test_heat_direction_is_unit_and_downhill(sphere):
    x, sten, W = sphere
    u = np.exp(-((x - x[0]) ** 2).sum(axis=1) / 0.1)
    eta = geodesic.heat_direction(W, sten, u)
    assert np.allclose(np.sqrt((eta * eta).sum(axis=1))[1:], 1.0)
    g = geodesic.gradient(W, sten, u)
    assert np.all((eta * g).sum(axis=1)[1:] < 0)


def test_heat_geodesic_approaches_great_circle_distance(sphere):
    x, sten, W = sphere
    wl = synth.geodesic_workload(4096)
    assert np.array_equal(wl.xyz, x)
    p = dict(wl.params)
    Hp = hierarchy.build(x, x, p)
    Hh = hierarchy.build(x, x, dict(p, problem="screened", mu=wl.heat["dt"]))
    src = wl.heat["source"]
    phi, iters = geodesic.heat_geodesic(Hh, Hp, W, sten, src, steps=wl.heat["steps"])
    d = np.arccos(np.clip(x @ x[src], -1.0, 1.0))
    assert phi[src] == 0.0
    assert np.mean(np.abs(phi - d)) < 0.04 and np.max(np.abs(phi - d)) < 0.08
    assert max(iters) <= 20
