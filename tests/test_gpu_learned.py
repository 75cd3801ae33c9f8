"""GPU learned smoother (training and inference kernels) against the oracle.

Tolerances: the device trains in FP32 (MLP, smoother adjoint, Adam) against
the oracle's FP64 maths on the same snapshots, so losses agree to ~1e-5 and
gradients to ~1e-4 relative (single-precision sums over 4k nodes and 8
snapshots); the weight initialisation is the same counter-based draw rounded
once to FP32 and must match bit for bit. With the step weights fixed, the
V-cycle is FP64 arithmetic on both sides (1e-10, as for Gauss-Seidel).
"""
import numpy as np
import pytest

import synth
from oracle import hierarchy, krylov, learned, precision, vcycle
from paper_2204_06154_amd import mgm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _flat(params):
    W1, b1, W2, b2, W3, b3 = params
    return np.concatenate([np.vstack([W1, b1[None]]).ravel(), np.vstack([W2, b2[None]]).ravel(),
                           np.vstack([W3, b3[None]]).ravel()])


CASES = {
    # jittered Fibonacci sphere N=4096, RBF-FD r^3 + deg 2, k=30 (screened)
    "sphere4096": lambda: synth.sphere_workload(4096),
    # the learned-smoother workload family at small N: star surface with 16:1
    # density bumps, RBF-FD r^3 + deg 2, k=30, screened
    "stardens6000": lambda: synth.star_density_workload(6000, n_probe=60_000),
}


@pytest.fixture(scope="module", params=list(CASES), ids=list(CASES))
def setup(request):
    wl = CASES[request.param]()
    print(f"[gpu-learned] setting up {request.param}", flush=True)
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=0)
    starts = np.random.default_rng(21).standard_normal((2, len(wl.xyz)))
    d_starts = torch.tensor(starts, device="cuda")
    info = m.train_smoother(d_starts, steps=0, s=3, iters_per_start=2, seed=9, init=True, activate=0)
    L = H.levels[0].L
    X = learned.stencil_features(H)
    S = learned.snapshots(H, starts, 2)
    yield wl, H, m, info, L, X, S, d_starts
    m.close()


def test_spectral_estimate_and_initialisation(setup):
    wl, H, m, info, L, X, S, _ = setup
    lam = learned.power_estimate(L)
    assert abs(info["lam"] - lam) <= 1e-10 * lam
    p0 = learned.init_params(X.shape[1], 3, seed=9)
    assert np.array_equal(m.smoother_params(), _flat(p0).astype(np.float32))


def test_forward_loss_and_gradient(setup):
    wl, H, m, info, L, X, S, _ = setup
    w = learned.cheb_omegas(info["lam"], 3)
    params = learned.init_params(X.shape[1], 3, seed=9)
    params[4] = 0.2 * np.random.default_rng(22).standard_normal(params[4].shape)
    params[5] = 0.1 * np.random.default_rng(23).standard_normal(params[5].shape)
    m.smoother_params(_flat(params))
    # step weights (MLP forward) against the oracle
    o, _ = learned.mlp_forward(params, X)
    om_ref = learned.omegas_from_output(o, w)
    om = m.export("omega").reshape(om_ref.shape)
    assert np.max(np.abs(om - om_ref)) <= 1e-5 * np.abs(om_ref).max()
    # loss and gradient
    loss, g = m.smoother_grad()
    loss_ref, grads = learned.total_loss_and_grads(params, X, L, S, w)
    g_ref = _flat(grads)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    for lo, hi in ((0, 91 * 64), (91 * 64, 91 * 64 + 65 * 64), (91 * 64 + 65 * 64, len(g_ref))):
        assert np.linalg.norm(g[lo:hi] - g_ref[lo:hi]) <= 1e-3 * np.linalg.norm(g_ref[lo:hi])


def test_vcycle_with_learned_smoother(setup):
    wl, H, m, info, L, X, S, _ = setup
    m.set_smoother(True)
    try:
        om = m.export("omega").reshape(-1, 3)
        ops = vcycle.Fp64Ops(H)
        ops.learned = om
        M = vcycle.make_preconditioner(ops, H.problem)
        z = m.vcycle(torch.tensor(wl.f, device="cuda")).cpu().numpy()
        zr = M(wl.f)
        assert np.max(np.abs(z - zr)) <= 1e-10 * np.abs(zr).max()
        A = vcycle.make_operator(H)
        _, info_ref = krylov.fgmres(A, M, wl.f, tol=1e-10, maxit=200)
        u, inf = m.solve(torch.tensor(wl.f, device="cuda"), rtol=1e-10, maxit=200)
        assert inf["status"] == 0 and inf["iters"] == info_ref.iters
        assert np.linalg.norm(wl.f - A(u.cpu().numpy())) <= 1.01e-10 * np.linalg.norm(wl.f)
    finally:
        m.set_smoother(False)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_reduced_precision_cycle_with_learned_smoother(setup, prec):
    """The reduced-precision V-cycle with the learned fine-level smoother
    against the oracle's emulation of that precision with the same step
    weights (1e-5, as for the Gauss-Seidel cycle)."""
    wl, H, m, info, L, X, S, _ = setup
    om = m.export("omega").reshape(-1, 3)
    m.set_smoother(True)
    m.set_precision(prec)
    try:
        ops = precision.ops_for(H, prec)
        ops.learned = om.astype(np.float32)
        z = m.vcycle(torch.tensor(wl.f, device="cuda")).cpu().numpy()
        ze = vcycle.make_preconditioner(ops, H.problem)(wl.f)
        assert np.linalg.norm(z - ze) / np.linalg.norm(ze) < 1e-5
    finally:
        m.set_precision("fp64")
        m.set_smoother(False)


def test_training_steps_follow_oracle(setup):
    wl, H, m, info, L, X, S, d_starts = setup
    w = learned.cheb_omegas(info["lam"], 3)
    params = learned.init_params(X.shape[1], 3, seed=9)
    m.smoother_params(_flat(params))
    res = m.train_smoother(None, steps=20, lr=1e-3, s=3, init=False, activate=0, history=True)
    _, hist_ref = learned.train(params, X, L, S, w, 20, lr=1e-3)
    hist = res["history"][:20]
    assert np.max(np.abs(hist - np.array(hist_ref)) / np.array(hist_ref)) < 1e-4
    assert res["loss_last"] < res["loss_first"]


def test_activation_with_fallback_rule(setup):
    wl, H, m, info, L, X, S, d_starts = setup
    res = m.train_smoother(d_starts, steps=40, lr=1e-3, s=3, iters_per_start=2, seed=9, init=True, activate=1)
    assert res["rate_gs"] > 0 and res["rate_learned"] > 0
    assert res["active"] == (res["rate_learned"] < res["rate_gs"])
    m.set_smoother(False)


def test_coarse_level_smoother_matches_oracle(setup):
    """Learned smoother on level 1 (its own features, spectral estimate,
    snapshots from the level-1 sub-cycle, loss and gradient), then the cycle
    with learned smoothing on levels 0 and 1 against the oracle."""
    wl, H, m, info, L0, X0, S0, _ = setup
    lv = H.levels[1]
    rng = np.random.default_rng(31)
    starts1 = rng.standard_normal((2, lv.N))
    info1 = m.train_smoother(torch.tensor(starts1, device="cuda"), steps=0, s=3, iters_per_start=2, seed=11,
                             init=True, activate=0, level=1)
    L1 = lv.L
    assert abs(info1["lam"] - learned.power_estimate(L1)) <= 1e-10 * info1["lam"]
    X1 = learned.level_features(H, 1)
    p1 = learned.init_params(X1.shape[1], 3, seed=11)
    assert np.array_equal(m.smoother_params(level=1), _flat(p1).astype(np.float32))
    w1 = learned.cheb_omegas(info1["lam"], 3)
    p1[4] = 0.2 * rng.standard_normal(p1[4].shape)
    p1[5] = 0.1 * rng.standard_normal(p1[5].shape)
    m.smoother_params(_flat(p1), level=1)
    o, _ = learned.mlp_forward(p1, X1)
    om1_ref = learned.omegas_from_output(o, w1)
    om1 = m.export("omega", 1).reshape(om1_ref.shape)
    assert np.max(np.abs(om1 - om1_ref)) <= 1e-5 * np.abs(om1_ref).max()
    S1 = learned.snapshots(H, starts1, 2, level=1)
    loss, g = m.smoother_grad(level=1)
    loss_ref, grads = learned.total_loss_and_grads(p1, X1, L1, S1, w1)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    assert np.linalg.norm(g - _flat(grads)) <= 1e-4 * np.linalg.norm(_flat(grads))
    # the cycle with learned smoothing on levels 0 and 1
    m.set_smoother(3)
    try:
        om0 = m.export("omega", 0).reshape(-1, 3)
        ops = vcycle.Fp64Ops(H)
        ops.learned = {0: om0, 1: om1}
        M = vcycle.make_preconditioner(ops, H.problem)
        z = m.vcycle(torch.tensor(wl.f, device="cuda")).cpu().numpy()
        zr = M(wl.f)
        assert np.max(np.abs(z - zr)) <= 1e-10 * np.abs(zr).max()
        A = vcycle.make_operator(H)
        _, info_ref = krylov.fgmres(A, M, wl.f, tol=1e-10, maxit=200)
        u, inf = m.solve(torch.tensor(wl.f, device="cuda"), rtol=1e-10, maxit=200)
        assert inf["status"] == 0 and inf["iters"] == info_ref.iters
        # only level 1
        m.set_smoother(2)
        ops.learned = {1: om1}
        z = m.vcycle(torch.tensor(wl.f, device="cuda")).cpu().numpy()
        zr = vcycle.make_preconditioner(ops, H.problem)(wl.f)
        assert np.max(np.abs(z - zr)) <= 1e-10 * np.abs(zr).max()
    finally:
        m.set_smoother(0)
    with pytest.raises(mgm.MgmError):
        m.set_smoother(4)   # level 2 has no trained smoother


def test_retraining_with_more_steps_per_sweep(setup):
    """Snapshots made with s = 2 are kept when the level is retrained with
    s = 5 and no new starts, so the adjoint's per-step buffers must grow with
    s: loss and gradient against the oracle on the same snapshots."""
    wl, H, m, info, L, X, S, d_starts = setup
    m.train_smoother(d_starts, steps=0, s=2, iters_per_start=2, seed=9, init=True, activate=0)
    res = m.train_smoother(None, steps=0, s=5, seed=9, init=True, activate=0)
    w = learned.cheb_omegas(res["lam"], 5)
    p = learned.init_params(X.shape[1], 5, seed=9)
    rng = np.random.default_rng(12)
    p[4] = 0.2 * rng.standard_normal(p[4].shape)
    m.smoother_params(_flat(p))
    loss, g = m.smoother_grad()
    loss_ref, grads = learned.total_loss_and_grads(p, X, L, S, w)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    assert np.linalg.norm(g - _flat(grads)) <= 1e-4 * np.linalg.norm(_flat(grads))
    res = m.train_smoother(None, steps=5, lr=1e-3, s=5, init=False, activate=0)
    assert res["loss_last"] < res["loss_first"]
