"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances. FP64: every kernel is the same arithmetic as the oracle in a
different summation order (and with fused multiply-adds), so single operator
applications agree to a few ulp of the row's magnitude (1e-13 relative). The
V-cycle chains ~10^2 such steps and a dense coarse inverse (vs. the oracle's
LU solve; the coarse operators have condition numbers up to ~1e5), so its
output is held to 1e-10 relative, and iteration counts must be identical.
These comparisons include the difference between the two FP64 setups (the
local weight solves round differently, ~1e-10 of a row's scale);
test_gpu_exported_parity.py runs the oracle on the library's own operators
and holds the V-cycle to 1e-12 and the Krylov iterates to 1e-10. FP32/FP16: compared with the oracle's emulation of
the same reduced-precision arithmetic (quantisation is bit-exact, so only
FP32 summation order differs): 1e-5 relative for a V-cycle. All solves must
reach a true FP64 relative residual of 1e-10.
"""
import numpy as np
import pytest

import synth
from oracle import hierarchy, krylov, precision, vcycle
from paper_2204_06154_amd import mgm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    # jittered Fibonacci sphere N=4096, RBF-FD r^3 + deg 2, k=30, screened mu=1
    "sphere4096": (lambda: synth.sphere_workload(4096), {}),
    # torus Poisson (bordered), RBF-FD r^5 + deg 3, k=50: the benchmark's torus family at small N
    "torus8000": (lambda: synth.torus_workload(8000), {"n_min": 250}),
    # GFD deg 2, k=25 on a ragged-size plain Fibonacci sphere (the 2^20-point sphere's family)
    "gfd9001": (lambda: synth.big_sphere_workload(9001), {"n_min": 150}),
    # plain multicolour GS (no patch blocking), bordered Poisson
    "torus6000plain": (lambda: synth.torus_workload(6000), {"n_min": 300, "gs_block": 0}),
}


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _rel_to(a, b, scale):
    """max |a - b| relative to the largest entry of a rounding-error scale
    (e.g. |L||x| for a product whose rows cancel, as Poisson rows do)."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(scale)), 1e-300))


@pytest.fixture(scope="module", params=list(CASES), ids=list(CASES))
def case(request):
    make, extra = CASES[request.param]
    wl = make()
    wl.params.update(extra)
    print(f"[gpu-parity] setting up {request.param}", flush=True)
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=0)
    yield request.param, wl, H, m
    m.close()


def _rhs(wl, H):
    return np.concatenate([wl.f, [0.0]]) if H.problem == "poisson" else wl.f.copy()


def test_device_handle_setup_matches_oracle(case):
    name, wl, H, m = case
    assert list(m.export("level_sizes")) == [lv.N for lv in H.levels]
    for j in range(len(H.levels) - 1):
        assert np.array_equal(m.export("colours", j), H.levels[j].colour)
        assert np.array_equal(m.export("coarse_idx", j), H.levels[j].coarse_idx)


def _exported_L(m, j, n):
    import scipy.sparse as sp
    return sp.csr_matrix((m.export("l_vals", j), m.export("l_cols", j), m.export("l_rowptr", j)), shape=(n, n))


def test_level_operators_fp64(case):
    """Against the oracle's operators. The library's FP64 setup values differ
    from the oracle's by the conditioning of the local solves (<= 1e-10 of the
    row scale, see the host tests), so products are compared relative to
    |L||x| at 1e-10; the kernel's own rounding is checked separately below."""
    name, wl, H, m = case
    m.set_precision("fp64")
    ops = vcycle.Fp64Ops(H)
    rng = np.random.default_rng(11)
    for j in range(len(H.levels) - 1):
        lv, nx = H.levels[j], H.levels[j + 1]
        x = rng.standard_normal(lv.N)
        b = rng.standard_normal(lv.N)
        # SpMV
        absLx = abs(lv.L) @ np.abs(x)
        y = _dev(np.zeros(lv.N))
        m.level_op(mgm.OP_SPMV, j, _dev(x), y=y)
        assert _rel_to(_host(y), lv.L @ x, absLx) < 1e-10, ("spmv", j)
        # GS sweeps (forward, backward; bordered with a multiplier)
        for rev in (False, True):
            lam = 0.3 if H.problem == "poisson" else 0.0
            xd = _dev(x)
            m.level_op(mgm.OP_SMOOTH, j, xd, b=_dev(b), scalar=lam, reverse=rev)
            ref = vcycle.gs_sweep(ops, j, x.copy(), b, lam, reverse=rev)
            scale = (np.abs(b) + abs(lv.L) @ np.abs(ref) + abs(lam)) / np.abs(lv.L.diagonal())
            assert _rel_to(_host(xd), ref, scale) < 1e-10, ("gs", j, rev)
        # residual + restriction
        yc = _dev(np.zeros(nx.N))
        m.level_op(mgm.OP_RESTRICT_RESIDUAL, j, _dev(x), b=_dev(b), y=yc)
        assert _rel_to(_host(yc), lv.R @ (b - lv.L @ x), abs(lv.R) @ (np.abs(b) + absLx)) < 1e-10, ("restrict", j)
        # interpolation + correction
        ec = rng.standard_normal(nx.N)
        xd = _dev(x)
        m.level_op(mgm.OP_INTERP_ADD, j, xd, y=_dev(ec))
        assert _rel(_host(xd), x + lv.P @ ec) < 1e-13, ("interp", j)


def test_spmv_kernel_rounding(case):
    """The device SpMV against the same (exported) FP64 operator on the host:
    only summation order differs, so |error| <= n eps |L||x| row by row."""
    name, wl, H, m = case
    m.set_precision("fp64")
    rng = np.random.default_rng(14)
    for j in range(len(H.levels) - 1):
        n = H.levels[j].N
        Lx = _exported_L(m, j, n)
        x = rng.standard_normal(n)
        y = _dev(np.zeros(n))
        m.level_op(mgm.OP_SPMV, j, _dev(x), y=y)
        width = np.diff(Lx.indptr)
        bound = width * np.finfo(float).eps * (abs(Lx) @ np.abs(x))
        assert np.all(np.abs(_host(y) - Lx @ x) <= bound), j


def test_vcycle_fp64_matches_oracle(case):
    name, wl, H, m = case
    m.set_precision("fp64")
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    rng = np.random.default_rng(12)
    for r in (_rhs(wl, H), rng.standard_normal(len(_rhs(wl, H)))):
        z = _host(m.vcycle(_dev(r)))
        assert _rel(z, M(r)) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_graph_replays_match_eager(case, prec):
    name, wl, H, m = case
    m.set_precision(prec)
    try:
        r = _dev(_rhs(wl, H))
        z_graph = []
        for _ in range(3):
            z_graph.append(_host(m.vcycle(r)))
            _host(m.apply(r))          # eager work between graph replays
        # a second handle without graphs gives the reference eager result
        p = dict(wl.params)
        p["use_graph"] = 0
        p["precision"] = prec
        m2 = mgm.Mgm(wl.xyz, wl.normals, p, device=0)
        z_eager = _host(m2.vcycle(r))
        for k, z in enumerate(z_graph):
            torch.cuda.synchronize()
            assert np.array_equal(z, z_eager), k
        m2.close()
    finally:
        m.set_precision("fp64")


@pytest.mark.parametrize("method", ["fgmres", "bicgstab"])
def test_solve_fp64_matches_oracle(case, method):
    name, wl, H, m = case
    m.set_precision("fp64")
    f = _rhs(wl, H)
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    solver = krylov.fgmres if method == "fgmres" else krylov.bicgstab
    x_ref, info_ref = solver(A, M, f, tol=1e-10, maxit=300)
    u, info = m.solve(_dev(f), krylov=method, restart=40, maxit=300, rtol=1e-10)
    u = _host(u)
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-10
    assert info["iters"] == info_ref.iters, (info["iters"], info_ref.iters)
    # the two solve systems whose operators differ by the setups' rounding
    # (~1e-10 of a row's scale), so their solutions differ by up to cond(A)
    # times that; iterates are compared on the library's own operators, to
    # 1e-10, in test_gpu_exported_parity.py
    # independent residual check with the oracle's operator
    assert np.linalg.norm(f - A(u)) <= 1.01e-10 * np.linalg.norm(f)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_reduced_precision_vcycle_matches_emulation(case, prec):
    name, wl, H, m = case
    m.set_precision(prec)
    try:
        f = _rhs(wl, H)
        Me = vcycle.make_preconditioner(precision.ops_for(H, prec), H.problem)
        M64 = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
        z = _host(m.vcycle(_dev(f)))
        ze = Me(f)
        assert np.linalg.norm(z - ze) / np.linalg.norm(ze) < 1e-5
        err64 = np.linalg.norm(z - M64(f)) / np.linalg.norm(M64(f))
        print(f"[{name}] {prec} V-cycle error vs FP64 oracle: {err64:.2e}")
        assert err64 < (1e-5 if prec == "fp32" else 5e-3)
    finally:
        m.set_precision("fp64")


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_reduced_precision_solve(case, prec):
    name, wl, H, m = case
    f = _rhs(wl, H)
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    _, info_ref = krylov.fgmres(A, M, f, tol=1e-10, maxit=300)
    m.set_precision(prec)
    try:
        u, info = m.solve(_dev(f), krylov="fgmres", restart=40, maxit=300, rtol=1e-10)
    finally:
        m.set_precision("fp64")
    u = _host(u)
    assert info["status"] == 0
    assert np.linalg.norm(f - A(u)) <= 1.01e-10 * np.linalg.norm(f)
    assert abs(info["iters"] - info_ref.iters) <= 1, (info["iters"], info_ref.iters)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_reduced_precision_bicgstab(case, prec):
    """The reduced-precision V-cycle inside BiCGSTAB (the 1M-point GFD sphere's
    solver): true FP64 residual 1e-10, applications within +-2 of the FP64
    oracle's (one BiCGSTAB step applies the preconditioner twice)."""
    name, wl, H, m = case
    f = _rhs(wl, H)
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    _, info_ref = krylov.bicgstab(A, M, f, tol=1e-10, maxit=300)
    m.set_precision(prec)
    try:
        u, info = m.solve(_dev(f), krylov="bicgstab", maxit=300, rtol=1e-10)
    finally:
        m.set_precision("fp64")
    u = _host(u)
    assert info["status"] == 0
    assert np.linalg.norm(f - A(u)) <= 1.01e-10 * np.linalg.norm(f)
    assert abs(info["iters"] - info_ref.iters) <= 2, (info["iters"], info_ref.iters)


@pytest.mark.parametrize("cycle,nu1,nu2,pre,post", [("V", 2, 2, "fwd", "fwd"), ("V", 1, 1, "fwd", "bwd"),
                                                     ("V", 0, 2, "fwd", "bwd"), ("V", 2, 0, "bwd", "fwd"),
                                                     ("W", 1, 1, "fwd", "fwd"), ("F", 1, 1, "fwd", "bwd")])
def test_cycle_variants_match_oracle(case, cycle, nu1, nu2, pre, post):
    """V/W/F(nu1, nu2) cycles with forward or backward sweeps (Sec. 4.3;
    symmetric GS = forward pre- and backward post-smoothing): the cycle to
    1e-10 and the FGMRES iteration count of the oracle with the same cycle."""
    name, wl, H, m = case
    p = dict(wl.params, nu1=nu1, nu2=nu2, pre_smoother=pre, post_smoother=post, cycle=cycle)
    mv = mgm.Mgm(wl.xyz, wl.normals, p, device=0)
    try:
        M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem, nu1, nu2, post_reverse=post == "bwd",
                                       pre_reverse=pre == "bwd", cycle=cycle)
        f = _rhs(wl, H)
        assert _rel(_host(mv.vcycle(_dev(f))), M(f)) < 1e-10
        A = vcycle.make_operator(H)
        _, info_ref = krylov.fgmres(A, M, f, tol=1e-10, maxit=300)
        u, info = mv.solve(_dev(f), krylov="fgmres", restart=40, maxit=300, rtol=1e-10)
        assert info["status"] == 0 and info["iters"] == info_ref.iters, (info["iters"], info_ref.iters)
        assert np.linalg.norm(f - A(_host(u))) <= 1.01e-10 * np.linalg.norm(f)
    finally:
        mv.close()


def test_warm_start_matches_oracle(case):
    """FGMRES from a caller-supplied initial guess (a perturbed solution, as
    a time-stepping solve would pass): the same iteration count as the
    oracle's FGMRES from the same guess."""
    name, wl, H, m = case
    m.set_precision("fp64")
    f = _rhs(wl, H)
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    x_ref, _ = krylov.fgmres(A, M, f, tol=1e-10, maxit=300)
    x0 = x_ref + 1e-4 * np.random.default_rng(16).standard_normal(len(f)) * np.abs(x_ref).max()
    _, info_ref = krylov.fgmres(A, M, f, tol=1e-10, maxit=300, x0=x0)
    u = _dev(x0)
    u, info = m.solve(_dev(f), u, krylov="fgmres", restart=40, maxit=300, rtol=1e-10, x0=True)
    assert info["status"] == 0 and info["iters"] == info_ref.iters, (info["iters"], info_ref.iters)
    assert np.linalg.norm(f - A(_host(u))) <= 1.01e-10 * np.linalg.norm(f)


def test_stationary_iteration_matches_oracle(case):
    name, wl, H, m = case
    m.set_precision("fp64")
    f = _rhs(wl, H)
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    u_ref = np.zeros_like(f)
    for _ in range(5):
        u_ref = u_ref + M(f - A(u_ref))
    u, info = m.solve(_dev(f), krylov="stationary", maxit=5, rtol=1e-30)
    assert info["status"] == 1 and info["iters"] == 5
    assert np.linalg.norm(_host(u) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def test_apply_matches_oracle(case):
    name, wl, H, m = case
    A = vcycle.make_operator(H)
    x = np.random.default_rng(13).standard_normal(len(_rhs(wl, H)))
    y = _host(m.apply(_dev(x)))
    L = H.levels[0].L
    scale = abs(L) @ np.abs(x[:L.shape[0]]) + np.abs(x).sum() * (H.problem == "poisson")
    assert _rel_to(y[:L.shape[0]], A(x)[:L.shape[0]], scale) < 1e-10
    if H.problem == "poisson":
        assert abs(y[-1] - A(x)[-1]) < 1e-13 * np.abs(x).sum()


def test_solver_error_paths(case):
    name, wl, H, m = case
    f = _rhs(wl, H)
    bad = f.copy()
    bad[7] = np.nan
    with pytest.raises(mgm.MgmError) as ei:
        m.solve(_dev(bad))
    assert ei.value.status == -9
    u, info = m.solve(_dev(f), maxit=1)
    assert info["status"] == 1 and info["iters"] == 1
    u, info = m.solve(_dev(np.zeros_like(f)))
    assert info["status"] == 0 and float(torch.abs(u).max()) == 0.0
    # the longest restart runs to its end (its last step's second projection
    # takes 201 dots) and reports "not converged" against an unreachable tolerance
    u, info = m.solve(_dev(f), restart=200, maxit=200, rtol=1e-30)
    assert info["status"] == 1 and info["iters"] == 200
    assert np.isfinite(_host(u)).all()


def test_time_kernel_modes(case):
    """Profiling entry point: every mode returns a positive time and the
    algorithmic bytes; the whole-V-cycle smoother batch averages per launch."""
    name, wl, H, m = case
    for which, level in (("spmv", 0), ("gs", 0), ("gs", -1), ("residual", 0), ("vcycle", 0)):
        ms, nbytes = m.time_kernel(which, level, reps=2)
        assert ms > 0.0 and nbytes > 0.0, (which, level)
    _, b_all = m.time_kernel("gs", -1, reps=1)
    _, b_v = m.time_kernel("vcycle", 0, reps=1)
    assert b_all < b_v

