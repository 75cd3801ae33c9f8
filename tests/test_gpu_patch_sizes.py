"""Patch-blocked Gauss-Seidel with patch sizes other than 256 against the
oracle: a ragged size that divides no level (37), a mid size (100) and the
degenerate one-point patches (1, where the patch graph is the point graph and
every patch has a single local colour), each with one launch per sweep and
with one launch per patch colour. The bordered Poisson torus runs with small
patches (16 and 37 points): its row operators then write two partial sums per
16 or 37 rows, more than the one per 16 rows of a plain level.

Tolerances as in test_gpu_parity: FP64 V-cycle output 1e-10 relative to the
oracle's (same arithmetic, different summation order and fused multiply-adds),
FGMRES iteration counts identical; the two launch modes bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import hierarchy, krylov, vcycle
from paper_2204_06154_amd import mgm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [("sphere", 4096, 37), ("sphere", 4096, 100), ("sphere", 1500, 1), ("torus", 6000, 16), ("torus", 6000, 37)]


@pytest.fixture(scope="module", params=CASES, ids=[f"{s}{n}_block{b}" for s, n, b in CASES])
def case(request):
    surf, n, block = request.param
    wl = synth.sphere_workload(n) if surf == "sphere" else synth.torus_workload(n)
    wl.params["gs_block"] = block
    print(f"[gpu-patch-sizes] setting up {surf} N={n} gs_block={block}", flush=True)
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    m1 = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, gs_flow=1), device=0)
    m0 = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, gs_flow=0), device=0)
    yield wl, H, m1, m0
    m1.close()
    m0.close()


def test_patches_follow_the_oracle(case):
    wl, H, m1, m0 = case
    for j in range(len(H.levels) - 1):
        assert np.array_equal(m1.export("patch", j), H.levels[j].patches["patch"]), j
        assert np.array_equal(m1.export("colours", j), H.levels[j].colour), j


def test_vcycle_and_solve_match_oracle(case):
    wl, H, m1, m0 = case
    ops = vcycle.Fp64Ops(H)
    M = vcycle.make_preconditioner(ops, H.problem)
    rhs = np.concatenate([wl.f, [0.0]]) if H.problem == "poisson" else wl.f
    zr = M(rhs)
    f = torch.tensor(rhs, device="cuda")
    z1 = m1.vcycle(f)
    z0 = m0.vcycle(f)
    torch.cuda.synchronize()
    assert torch.equal(z1, z0)
    z = z1.cpu().numpy()
    assert np.max(np.abs(z - zr)) <= 1e-10 * np.abs(zr).max()
    A = vcycle.make_operator(H)
    _, info_ref = krylov.fgmres(A, M, rhs, tol=1e-10, maxit=200)
    u, info = m1.solve(f, rtol=1e-10, maxit=200)
    assert info["status"] == 0 and info["iters"] == info_ref.iters
    assert np.linalg.norm(rhs - A(u.cpu().numpy())) <= 1.01e-10 * np.linalg.norm(rhs)
