"""The paper's scaling-study problem on the GPU (Table 2 setting).

Icosahedral sphere nodes (N = 10,242), shifted Poisson (mu = 1) with a random
right-hand side, RBF-FD l = 3 and l = 7 (PHS order k = l, n = (l+1)(l+2)),
FGMRES(40) and BiCGSTAB with the FP64 cycle to 1e-12: the device takes the
oracle's iteration counts and reaches the true residual.
"""
import numpy as np
import pytest

import synth
from oracle import hierarchy, krylov, vcycle
from paper_2204_06154_amd import mgm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


# The degree-7 (PHS r^15) stencil systems reach cond ~2.5e11, so the
# library's weights and the oracle's differ by ~1e-9 relative: the solution
# meets 1e-12 against the library's own operator and ~1e-9 against the oracle's.
ORACLE_RES = {3: 1.01e-12, 7: 1e-8}


@pytest.mark.parametrize("ell", [3, 7])
def test_icosahedral_solves_match_oracle(ell):
    wl = synth.icosahedral_workload(5, ell)
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    A = vcycle.make_operator(H)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H), H.problem)
    _, ig = krylov.fgmres(A, M, wl.f, tol=1e-12, restart=40, maxit=200)
    _, ib = krylov.bicgstab(A, M, wl.f, tol=1e-12, maxit=200)
    m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=0)
    try:
        f = torch.tensor(wl.f, device="cuda")
        for kry, ref in (("fgmres", ig), ("bicgstab", ib)):
            u, info = m.solve(f, krylov=kry, restart=40, maxit=200, rtol=1e-12)
            assert info["status"] == 0 and info["iters"] == ref.iters, (kry, info["iters"], ref.iters)
            own = (f - m.apply(u)).cpu().numpy()
            assert np.linalg.norm(own) <= 1.01e-12 * np.linalg.norm(wl.f)
            assert np.linalg.norm(wl.f - A(u.cpu().numpy())) <= ORACLE_RES[ell] * np.linalg.norm(wl.f)
    finally:
        m.close()
