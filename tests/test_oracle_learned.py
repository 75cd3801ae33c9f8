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


# ------------------------------------------- bordered Poisson system (Sec. 4.4)
@pytest.fixture(scope="module")
def torus_small():
    wl = synth.torus_workload(1500)
    wl.params["n_min"] = 60
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    assert H.problem == "poisson" and len(H.levels) >= 3
    return wl, H


def _weights(N, s, seed):
    rng = np.random.default_rng(seed)
    return 0.4 + 0.6 * rng.random((N, s))


def _step_product(L, omega, left):
    """prod_q (I - W_q L) (left=False) or prod_q (I - L W_q) (left=True),
    W_q = diag(omega_q / L_ii), later steps on the left."""
    N = L.shape[0]
    E = np.eye(N)
    for q in range(omega.shape[1]):
        W = np.diag(omega[:, q] / np.diag(L))
        E = ((np.eye(N) - L @ W) if left else (np.eye(N) - W @ L)) @ E
    return E


@pytest.mark.parametrize("j", [0, 1])
def test_bordered_learned_sweep_holds_the_multiplier(torus_small, j):
    """With the multiplier fixed at lam, every v with L_j v + b_j lam = f is a
    fixed point and the error propagates by the dense product
    prod_q (I - W_q L_j): u_s - v = E (u_0 - v)."""
    _, H = torus_small
    lv = H.levels[j]
    L = lv.L.toarray()
    rng = np.random.default_rng(40 + j)
    v = rng.standard_normal(lv.N)
    lam = 0.7
    f = L @ v + lv.b * lam
    omega = _weights(lv.N, 3, 41 + j)
    ops = vcycle.Fp64Ops(H)
    ops.learned = {j: omega}
    u0 = rng.standard_normal(lv.N)
    u = vcycle.learned_sweep(ops, u0.copy(), f, j, lam)
    ref = v + _step_product(L, omega, False) @ (u0 - v)
    assert np.allclose(u, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_bordered_cycle_post_smoothing_uses_the_coarse_multiplier(torus_small):
    """Bordered V-cycle with learned smoothing on levels 0 and 1: with e_c the
    level-0 vector right after the coarse correction and mu the multiplier
    correction the cycle returns, the post-smoothed residual is
    prod_q (I - L W_q) (r - L e_c - b mu) (the smoother holds mu fixed)."""
    _, H = torus_small
    lv = H.levels[0]
    L = lv.L.toarray()
    ops = vcycle.Fp64Ops(H)
    ops.learned = {0: _weights(lv.N, 3, 50), 1: _weights(H.levels[1].N, 2, 51)}
    rng = np.random.default_rng(52)
    r, rho = rng.standard_normal(lv.N), 0.3
    cap = []
    z, mu = vcycle.vcycle(ops, r, rho, capture=cap)
    assert abs(mu) > 1e-3
    r_mid = r - L @ cap[0] - lv.b * mu
    ref = _step_product(L, ops.learned[0], True) @ r_mid
    out = r - L @ z - lv.b * mu
    assert np.allclose(out, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_bordered_two_level_cycle_by_definition():
    """Two levels, learned smoothing on level 0, V(1,1): z = e_1 + P e_c + post,
    with e_1 the s steps from zero (no multiplier), (e_c, mu) the exact solution
    of the coarse bordered system [L_c b_c; b_c^T 0] for (R(r - L e_1),
    rho - b . e_1), and the post-smoother's s steps with mu fixed; every step
    written as a dense affine map."""
    wl = synth.torus_workload(700)
    wl.params["n_min"] = 100
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    assert len(H.levels) == 2
    lv, cl = H.levels
    L, P, R = lv.L.toarray(), lv.P.toarray(), lv.R.toarray()
    Lc, bc, b = cl.L.toarray(), cl.b, lv.b
    N = lv.N
    omega = _weights(N, 3, 60)
    rng = np.random.default_rng(61)
    r, rho = rng.standard_normal(N), -0.4
    # s steps from zero: u_s = G r, G = sum_q (prod_{p>q} (I - W_p L)) W_q
    Ws = [np.diag(omega[:, q] / np.diag(L)) for q in range(3)]
    G = np.zeros((N, N))
    for q in range(3):
        G = (np.eye(N) - Ws[q] @ L) @ G + Ws[q]
    e1 = G @ r
    K = np.block([[Lc, bc[:, None]], [bc[None, :], np.zeros((1, 1))]])
    sol = np.linalg.solve(K, np.concatenate([R @ (r - L @ e1), [rho - b @ e1]]))
    e2, mu = e1 + P @ sol[:-1], sol[-1]
    z_ref = e2 + G @ (r - L @ e2 - b * mu)
    ops = vcycle.Fp64Ops(H)
    ops.learned = omega
    z, mu_o = vcycle.vcycle(ops, r, rho)
    assert abs(mu_o - mu) <= 1e-10 * abs(mu)
    assert np.allclose(z, z_ref, rtol=0, atol=1e-10 * np.abs(z_ref).max())


def test_bordered_snapshots_follow_the_bordered_iteration(torus_small):
    """Bordered snapshots: the iterate x = (e, mu) follows x <- x + M(-A x)
    with the bordered operator and preconditioner (from (start, 0)); each
    snapshot is e + the level-0 vector captured right after the coarse
    correction of the cycle applied to -A x."""
    _, H = torus_small
    lv = H.levels[0]
    rng = np.random.default_rng(70)
    e0 = rng.standard_normal(lv.N)
    S = learned.snapshots(H, e0[None, :], 3)
    ops = vcycle.Fp64Ops(H)
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(ops, H.problem)
    x = np.concatenate([e0, [0.0]])
    for t in range(3):
        ax = A(x)
        cap = []
        vcycle.vcycle(ops, -ax[:-1], -ax[-1], capture=cap)
        assert np.allclose(S[t], x[:-1] + cap[0], rtol=0, atol=1e-10 * np.abs(S[t]).max())
        x = x + M(-ax)
        if t == 0:
            assert abs(x[-1]) > 1e-6          # later iterations carry a multiplier


def test_bordered_omega_gradient_matches_finite_differences(torus_small):
    """The loss on bordered snapshots (the torus Laplacian, singular) and its
    adjoint gradient against central differences."""
    _, H = torus_small
    L = H.levels[0].L
    S = learned.snapshots(H, np.random.default_rng(80).standard_normal((2, L.shape[0])), 2)
    rng = np.random.default_rng(81)
    omega = 0.5 + 0.3 * rng.random((L.shape[0], 3))
    loss, g = learned.loss_and_grad_omega(L, omega, S)
    for _ in range(10):
        i, q = rng.integers(L.shape[0]), rng.integers(3)
        h = 1e-4                          # loss ~1e-2: smaller steps drown in rounding
        op, om = omega.copy(), omega.copy()
        op[i, q] += h
        om[i, q] -= h
        fd = (learned.loss_and_grad_omega(L, op, S)[0] - learned.loss_and_grad_omega(L, om, S)[0]) / (2 * h)
        assert abs(fd - g[i, q]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max())


def test_mlp_forward_reduces_to_affine_maps():
    """Where no ReLU is active the network is one affine map,
    x -> x (W1 W2 W3) + (b1 W2 W3 + b2 W3 + b3) (the weight product formed
    first); where the first layer is switched off by its bias, the output
    is relu(b2) W3 + b3 whatever the input."""
    rng = np.random.default_rng(90)
    n_in, s = 12, 3
    W1, W2, W3 = rng.random((n_in, 64)), rng.random((64, 64)), rng.standard_normal((64, s))
    b1, b2, b3 = rng.random(64), rng.random(64), rng.standard_normal(s)
    X = rng.random((7, n_in))
    o, _ = learned.mlp_forward([W1, b1, W2, b2, W3, b3], X)
    Wp = W1 @ (W2 @ W3)
    bp = (b1 @ W2) @ W3 + b2 @ W3 + b3
    assert np.allclose(o, X @ Wp + bp, rtol=1e-12, atol=1e-12 * np.abs(o).max())
    b1_off = -1.0 - X.max() * np.abs(W1).sum(axis=0)          # every first-layer unit negative
    b2_mixed = rng.standard_normal(64)
    o2, _ = learned.mlp_forward([W1, b1_off, W2, b2_mixed, W3, b3], X)
    ref = np.maximum(b2_mixed, 0.0) @ W3 + b3
    assert np.allclose(o2, np.broadcast_to(ref, o2.shape), rtol=0, atol=1e-12)


def test_step_weights_stay_within_half_of_chebyshev():
    """omega = omega_q (1 + tanh(o) / 2): the Chebyshev weight at o = 0, its
    limits 1.5 and 0.5 times it for o -> +-inf, 1.25 times it at
    o = artanh(1/2)."""
    w = learned.cheb_omegas(2.0, 3)
    o = np.array([[0.0, 60.0, -60.0], [math.atanh(0.5), 0.0, 0.0]])
    om = learned.omegas_from_output(o, w)
    assert np.allclose(om[0], w * np.array([1.0, 1.5, 0.5]), rtol=1e-15)
    assert np.allclose(om[1], w * np.array([1.25, 1.0, 1.0]), rtol=1e-15)
