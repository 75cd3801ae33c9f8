"""Full-size parity on the benchmark workload, in the configuration bench.py times.

Torus R=1, r=1/3, N=160,000 Poisson-disk points, RBF-FD r^5 + degree 3 on
50-point stencils, bordered surface Poisson, patch-blocked GS (256-point
patches), HIP graphs on. The oracle builds its own hierarchy at this size
(about a minute on the host) and everything it produces is compared:

- the integer setup (level sizes, coarse subsets, colours, patches) bit for bit;
- one FP64 V-cycle (1e-10 relative, as at small sizes);
- the FP32 V-cycle against the oracle's FP32 emulation (1e-5 relative);
- the FP32-V-cycle FGMRES solve: the oracle's FP64 iteration count (within
  the +-1 allowed for reduced precision), and a true relative residual of
  1e-10 computed with the oracle's operator.
"""
import numpy as np
import pytest

import synth
from oracle import hierarchy, krylov, precision, vcycle
from paper_2204_06154_amd import mgm

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def torus():
    wl = synth.torus_workload(160_000)
    print("[fullsize] oracle setup, N=160000", flush=True)
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    print("[fullsize] library setup", flush=True)
    m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=0)
    yield wl, H, m
    m.close()


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_fullsize_setup_bit_exact(torus):
    wl, H, m = torus
    assert list(m.export("level_sizes")) == [lv.N for lv in H.levels] == [160000, 40000, 10000, 2500, 625]
    for j, lv in enumerate(H.levels[:-1]):
        assert np.array_equal(m.export("coarse_idx", j), lv.coarse_idx), j
        assert np.array_equal(m.export("colours", j), lv.colour), j
        assert np.array_equal(m.export("patch", j), lv.patches["patch"]), j


def test_fullsize_vcycles(torus):
    wl, H, m = torus
    f = np.concatenate([wl.f, [0.0]])
    m.set_precision("fp64")
    z64 = _host(m.vcycle(_dev(f)))
    ref64 = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)(f)
    assert np.max(np.abs(z64 - ref64)) <= 1e-10 * np.max(np.abs(ref64))
    m.set_precision("fp32")
    try:
        z32 = _host(m.vcycle(_dev(f)))
    finally:
        m.set_precision("fp64")
    ref32 = vcycle.make_preconditioner(precision.ops_for(H, "fp32"), H.problem)(f)
    assert np.linalg.norm(z32 - ref32) <= 1e-5 * np.linalg.norm(ref32)


def test_fullsize_fp32_solve(torus):
    wl, H, m = torus
    f = np.concatenate([wl.f, [0.0]])
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    _, info_ref = krylov.fgmres(A, M, f, tol=1e-10, restart=40, maxit=400)
    m.set_precision("fp32")
    try:
        u, info = m.solve(_dev(f), krylov="fgmres", restart=40, maxit=400, rtol=1e-10)
    finally:
        m.set_precision("fp64")
    u = _host(u)
    assert info["status"] == 0
    assert abs(info["iters"] - info_ref.iters) <= 1, (info["iters"], info_ref.iters)
    assert np.linalg.norm(f - A(u)) <= 1.01e-10 * np.linalg.norm(f)


def test_fullsize_learned_smoothers(torus):
    """The bench's learned configuration at full size: every smoothed level
    trains its network on the GPU (bordered, s = 2, 400 Adam steps at 3e-3)
    and keeps it if its factor beats Gauss-Seidel's. With the exported step
    weights, the FP64 cycle matches the oracle's to 1e-10 and the FP32 cycle
    the oracle's FP32 emulation to 1e-5; the FP32 FGMRES solve reaches a true
    relative residual of 1e-10 within one iteration of the oracle's FP64
    count with the same smoothers."""
    wl, H, m = torus
    f = np.concatenate([wl.f, [0.0]])
    sizes = [lv.N for lv in H.levels]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2204)
    mask = 0
    for j in range(len(sizes) - 1):
        sj = torch.randn((4, sizes[j]), generator=gen, device="cuda", dtype=torch.float64)
        t = m.train_smoother(sj, steps=400, lr=3e-3, s=2, iters_per_start=2, seed=5 + j, init=True, activate=1,
                             level=j)
        print(f"[fullsize] level {j}: factor GS {t['rate_gs']:.4f}, learned {t['rate_learned']:.4f}", flush=True)
        mask |= (1 << j) if t["active"] else 0
    assert mask != 0
    m.set_smoother(mask)
    try:
        om = {j: m.export("omega", j).reshape(sizes[j], -1) for j in range(len(sizes) - 1) if (mask >> j) & 1}
        ops = vcycle.Fp64Ops(H)
        ops.learned = om
        M = vcycle.make_preconditioner(ops, H.problem)
        m.set_precision("fp64")
        z64 = _host(m.vcycle(_dev(f)))
        ref64 = M(f)
        assert np.max(np.abs(z64 - ref64)) <= 1e-10 * np.max(np.abs(ref64))
        ops32 = precision.ops_for(H, "fp32")
        ops32.learned = {j: w.astype(np.float32) for j, w in om.items()}
        m.set_precision("fp32")
        z32 = _host(m.vcycle(_dev(f)))
        ref32 = vcycle.make_preconditioner(ops32, H.problem)(f)
        assert np.linalg.norm(z32 - ref32) <= 1e-5 * np.linalg.norm(ref32)
        A = vcycle.make_operator(H)
        _, info_ref = krylov.fgmres(A, M, f, tol=1e-10, restart=40, maxit=400)
        u, info = m.solve(_dev(f), krylov="fgmres", restart=40, maxit=400, rtol=1e-10)
        print(f"[fullsize] learned mask {mask:#x}: FGMRES {info['iters']} (oracle {info_ref.iters})", flush=True)
        assert info["status"] == 0 and abs(info["iters"] - info_ref.iters) <= 1, (info["iters"], info_ref.iters)
        assert np.linalg.norm(f - A(_host(u))) <= 1.01e-10 * np.linalg.norm(f)
    finally:
        m.set_precision("fp64")
        m.set_smoother(False)
