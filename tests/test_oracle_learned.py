"""Pins of the oracle's learned-smoother maths (an extension; our reading)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import chebyshev

import synth
from oracle import hierarchy, learned, vcycle


@pytest.fixture(scope="module")
def small():
    wl = synth.sphere_workload(700)
    wl.params["n_coarse_max"] = 120
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    X = learned.stencil_features(H)
    rng = np.random.default_rng(3)
    S = learned.snapshots(H, rng.standard_normal((2, H.levels[0].N)), 1)
    return H, X, S


def test_zero_last_layer_is_textbook_chebyshev():
    """s Richardson steps with omega_q = 1/theta_q (roots of the scaled Chebyshev
    polynomial on [a, b]) multiply an eigenvector of D^-1 L with eigenvalue lam
    by T_s((b + a - 2 lam)/(b - a)) / T_s((b + a)/(b - a))."""
    n, s = 40, 3
    L = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    lam_max = 1.0 - math.cos(n * math.pi / (n + 1))          # largest eigenvalue of D^-1 L = L/2
    w = learned.cheb_omegas(lam_max, s)
    params = learned.init_params(10, s, seed=1)
    o, _ = learned.mlp_forward(params, np.random.default_rng(0).standard_normal((n, 10)))
    assert np.all(o == 0.0)
    omega = learned.omegas_from_output(o, w)
    assert np.allclose(omega, w[None, :])
    a, b = lam_max / 4, 1.1 * lam_max
    Ts = np.zeros(s + 1)
    Ts[s] = 1.0
    for k in (3, 17, 40):
        v = np.sin(k * math.pi * np.arange(1, n + 1) / (n + 1))
        lam = 1.0 - math.cos(k * math.pi / (n + 1))
        out = learned.smooth(L, omega, v.copy())
        ref = chebyshev.chebval((b + a - 2 * lam) / (b - a), Ts) / chebyshev.chebval((b + a) / (b - a), Ts)
        assert np.allclose(out, ref * v, atol=1e-12)


def test_omega_gradient_matches_finite_differences(small):
    H, X, S = small
    L = H.levels[0].L
    rng = np.random.default_rng(4)
    omega = 0.5 + 0.3 * rng.random((L.shape[0], 3))
    loss, g = learned.loss_and_grad_omega(L, omega, S)
    for _ in range(12):
        i, q = rng.integers(L.shape[0]), rng.integers(3)
        h = 1e-6
        op, om = omega.copy(), omega.copy()
        op[i, q] += h
        om[i, q] -= h
        fd = (learned.loss_and_grad_omega(L, op, S)[0] - learned.loss_and_grad_omega(L, om, S)[0]) / (2 * h)
        assert abs(fd - g[i, q]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max())


def test_parameter_gradient_matches_finite_differences(small):
    H, X, S = small
    L = H.levels[0].L
    w = learned.cheb_omegas(learned.power_estimate(L), 3)
    params = learned.init_params(X.shape[1], 3, seed=5)
    rng = np.random.default_rng(6)
    params[4] = 0.1 * rng.standard_normal(params[4].shape)    # non-zero last layer: gradients reach W1, W2
    loss, grads = learned.total_loss_and_grads(params, X, L, S, w)
    for layer in range(6):
        for _ in range(3):
            idx = tuple(rng.integers(d) for d in params[layer].shape)
            h = 1e-6
            pp = [p.copy() for p in params]
            pm = [p.copy() for p in params]
            pp[layer][idx] += h
            pm[layer][idx] -= h
            fd = (learned.total_loss_and_grads(pp, X, L, S, w)[0] - learned.total_loss_and_grads(pm, X, L, S, w)[0]) / (2 * h)
            scale = max(abs(fd), 1e-4 * max(np.abs(g).max() for g in grads))
            assert abs(fd - grads[layer][idx]) <= 2e-6 * scale, (layer, idx, fd, grads[layer][idx])


def test_power_estimate_close_to_largest_eigenvalue(small):
    H, X, S = small
    L = H.levels[0].L
    M = sp.diags(1.0 / L.diagonal()) @ L
    ev = spla.eigs(M, k=1, which="LM", return_eigenvectors=False)
    lam = learned.power_estimate(L)
    assert abs(lam - abs(ev[0])) <= 0.1 * abs(ev[0])


def test_counter_generator_uses_splitmix64():
    from oracle import colouring
    keys = np.array([0, 1, 12345], dtype=np.uint64)
    u = learned.counter_uniform(keys)
    ref = (colouring.splitmix64(keys) >> np.uint64(11)).astype(np.float64) / 2.0 ** 53
    assert np.array_equal(u, ref) and np.all((u >= 0) & (u < 1))


def test_capture_is_state_after_coarse_correction():
    """Two-level: the captured vector equals u1 + P L_H^-1 R (r - L u1), u1 the pre-smoothed iterate."""
    wl = synth.sphere_workload(600)
    wl.params["n_coarse_max"] = 160
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    assert len(H.levels) == 2
    lv = H.levels[0]
    ops = vcycle.Fp64Ops(H)
    r = np.random.default_rng(7).standard_normal(lv.N)
    u1 = vcycle.gs_sweep(ops, 0, np.zeros(lv.N), r)
    P = lv.P.toarray()
    L = lv.L.toarray()
    ref = u1 + P @ np.linalg.solve(P.T @ L @ P, P.T @ (r - L @ u1))
    cap = []
    vcycle.vcycle(ops, r, None, capture=cap)
    assert np.allclose(cap[0], ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_training_reduces_the_loss(small):
    H, X, S = small
    L = H.levels[0].L
    w = learned.cheb_omegas(learned.power_estimate(L), 3)
    params = learned.init_params(X.shape[1], 3, seed=8)
    _, hist = learned.train(params, X, L, S, w, 30, lr=1e-3)
    assert hist[-1] < hist[0]


def test_coarse_level_features_by_definition(small):
    """Level-1 features: the n nearest level-1 points (brute force), their
    tangent-plane offsets over the stencil radius, and L_1 entries over the
    diagonal (0 off the pattern)."""
    from oracle import discretize
    H = small[0]
    X1 = learned.level_features(H, 1)
    lv = H.levels[1]
    n = min(H.stencils.shape[1], lv.N)
    assert X1.shape == (lv.N, 3 * n)
    fidx = learned.level_fine_index(H, 1)
    assert np.array_equal(H.levels[0].xyz[fidx], lv.xyz)
    L1 = lv.L.toarray()
    t1, t2 = discretize.tangent_frames(H.normals[fidx])
    for i in (0, 7, lv.N - 1):
        d = lv.xyz - lv.xyz[i]
        d2 = ((d[:, 0] * d[:, 0]) + (d[:, 1] * d[:, 1])) + d[:, 2] * d[:, 2]
        sten = np.lexsort((np.arange(lv.N), d2))[:n]
        xh = np.stack([d[sten] @ t1[i], d[sten] @ t2[i]], axis=1)
        rho = np.sqrt((xh ** 2).sum(axis=1)).max()
        assert np.allclose(X1[i, :2 * n], (xh / rho).ravel(), atol=1e-12)
        assert np.allclose(X1[i, 2 * n:], L1[i, sten] / abs(L1[i, i]), atol=1e-12)
    assert np.allclose(learned.level_features(H, 0), learned.stencil_features(H))


def test_coarse_level_snapshots_follow_sub_cycle(small):
    """Level-1 snapshots: e + (level-1 vector right after the coarse
    correction) of the level-1 sub-cycle; for a two-level sub-hierarchy (level
    2 coarsest) that vector is e_pre + P_1 L_2^-1 R_1 (f - L_1 e_pre), with
    e_pre the pre-smoothed iterate."""
    H = small[0]
    if len(H.levels) != 3:
        pytest.skip("needs exactly three levels")
    lv, cl = H.levels[1], H.levels[2]
    rng = np.random.default_rng(5)
    e0 = rng.standard_normal(lv.N)
    snap = learned.snapshots(H, e0[None, :], 1, level=1)[0]
    f = -(lv.L @ e0)
    ops = vcycle.Fp64Ops(H)
    u = vcycle.gs_sweep(ops, 1, np.zeros(lv.N), f)
    cap = u + lv.P @ np.linalg.solve(cl.L.toarray(), lv.R @ (f - lv.L @ u))
    assert np.allclose(snap, e0 + cap, rtol=0, atol=1e-10 * np.abs(e0 + cap).max())
