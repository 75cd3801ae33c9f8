"""The hot-path kernels against the oracle on the library's own operators.

The library and the oracle build their FP64 setups separately; their local
weight solves differ by the conditioning of those systems (~1e-10 of a row's
scale), and that difference, not the kernels, dominates a comparison of the
two end to end. Here the oracle's V-cycle and FGMRES run on the operators the
library exports (L_j, P_j, R_j = P_j^T, b_j and the coarsest operator; the
colourings are the oracle's own, which equal the library's bit for bit), so
what remains is the kernels' arithmetic: the same sums in another order, with
fused multiply-adds, and the coarsest solve by a dense inverse instead of an
LU solve.

Tolerances. A GS sweep, residual or transfer agrees to a few ulp of its
row's magnitude; the coarsest correction differs by ~cond(L_p)*eps relative
to itself, about 1e-12 for these coarse operators, and the smoothed levels
then damp, not amplify, that difference. The V-cycle output is held to 1e-12
relative. FGMRES iterates are held to 1e-10 relative with identical
iteration counts.

FP16 row-scale quantisation (h_ij = fp16(L_ij / s_i), s_i = fp32(max_j
|L_ij|), each rounded once from FP64 with round-to-nearest-even): the values
the device holds must equal NumPy's conversions of the exported FP64
operator bit for bit.
"""
import copy

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import synth
from oracle import hierarchy, krylov, vcycle
from paper_2204_06154_amd import mgm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "sphere4096": (lambda: synth.sphere_workload(4096), {}),
    "torus8000": (lambda: synth.torus_workload(8000), {"n_min": 250}),
    "gfd9001": (lambda: synth.big_sphere_workload(9001), {"n_min": 150}),
    "torus6000plain": (lambda: synth.torus_workload(6000), {"n_min": 300, "gs_block": 0}),
}


@pytest.fixture(scope="module", params=list(CASES), ids=list(CASES))
def case(request):
    make, extra = CASES[request.param]
    wl = make()
    wl.params.update(extra)
    print(f"[gpu-exported] setting up {request.param}", flush=True)
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=0)
    yield request.param, wl, H, m
    m.close()


def _exported_L(m, j, n):
    return sp.csr_matrix((m.export("l_vals", j), m.export("l_cols", j), m.export("l_rowptr", j)), shape=(n, n))


def _on_exported(H, m):
    """A copy of the oracle's hierarchy whose operators are the library's."""
    H2 = copy.copy(H)
    H2.levels = [copy.copy(lv) for lv in H.levels]
    p = len(H2.levels)
    for j, lv in enumerate(H2.levels):
        lv.L = _exported_L(m, j, lv.N)
        if H.problem == "poisson":
            lv.b = m.export("border", j)
        if j < p - 1:
            nc = H2.levels[j + 1].N
            idx = m.export("interp_idx", j).reshape(lv.N, -1)
            w = m.export("interp_w", j).reshape(lv.N, -1)
            rows = np.repeat(np.arange(lv.N), idx.shape[1])
            lv.P = sp.csr_matrix((w.ravel(), (rows, idx.ravel())), shape=(lv.N, nc))
            lv.R = lv.P.T.tocsr()
    Lp = H2.levels[-1].L.toarray()
    if H.problem == "poisson":
        b = H2.levels[-1].b
        n = len(b)
        Mb = np.zeros((n + 1, n + 1))
        Mb[:n, :n] = Lp
        Mb[:n, n] = b
        Mb[n, :n] = b
        H2.coarse_lu = sla.lu_factor(Mb)
    else:
        H2.coarse_lu = sla.lu_factor(Lp)
    return H2


def _rhs(wl, H):
    return np.concatenate([wl.f, [0.0]]) if H.problem == "poisson" else wl.f.copy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_exported_operators_equal_the_oracles_to_setup_rounding(case):
    """Sanity of the comparison: the exported operators are the oracle's up
    to the rounding of the separate setups."""
    name, wl, H, m = case
    H2 = _on_exported(H, m)
    for lv, lv2 in zip(H.levels, H2.levels):
        assert np.array_equal(lv.L.indptr, lv2.L.indptr) and np.array_equal(lv.L.indices, lv2.L.indices)
        assert np.max(np.abs(lv.L.data - lv2.L.data)) <= 1e-9 * np.max(np.abs(lv.L.data))


def test_vcycle_on_exported_operators(case):
    name, wl, H, m = case
    m.set_precision("fp64")
    H2 = _on_exported(H, m)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H2), H2.problem)
    rng = np.random.default_rng(21)
    f = _rhs(wl, H)
    for r in (f, rng.standard_normal(len(f))):
        z = m.vcycle(torch.tensor(r, device="cuda")).cpu().numpy()
        err = _rel(z, M(r))
        print(f"[gpu-exported] {name}: V-cycle rel. difference {err:.2e}", flush=True)
        assert err <= 1e-12


def test_fgmres_on_exported_operators(case):
    name, wl, H, m = case
    m.set_precision("fp64")
    H2 = _on_exported(H, m)
    A = vcycle.make_operator(H2)
    M = vcycle.make_preconditioner(vcycle.Fp64Ops(H2), H2.problem)
    f = _rhs(wl, H)
    x_ref, info_ref = krylov.fgmres(A, M, f, tol=1e-10, maxit=300)
    u, info = m.solve(torch.tensor(f, device="cuda"), krylov="fgmres", restart=40, maxit=300, rtol=1e-10)
    u = u.cpu().numpy()
    err = float(np.linalg.norm(u - x_ref) / np.linalg.norm(x_ref))
    print(f"[gpu-exported] {name}: FGMRES {info['iters']} iterations (oracle {info_ref.iters}), "
          f"iterate rel. difference {err:.2e}", flush=True)
    assert info["status"] == 0 and info["iters"] == info_ref.iters
    assert err <= 1e-10


def test_fp16_quantisation_is_bit_exact(case):
    name, wl, H, m = case
    for j in range(len(H.levels) - 1):
        L = _exported_L(m, j, H.levels[j].N)
        h = m.export("l16_vals", j)
        s = m.export("row_scale", j)
        rows = np.repeat(np.arange(L.shape[0]), np.diff(L.indptr))
        absmax = np.zeros(L.shape[0])
        np.maximum.at(absmax, rows, np.abs(L.data))
        s_ref = absmax.astype(np.float32)
        s_ref[s_ref == 0] = np.float32(1.0)
        h_ref = (L.data / s_ref.astype(np.float64)[rows]).astype(np.float16)
        assert np.array_equal(s.astype(np.float32).view(np.uint32), s_ref.view(np.uint32)), j
        assert np.array_equal(s, s_ref.astype(np.float64)), j  # the export widened exactly
        assert np.array_equal(h.astype(np.float16).view(np.uint16), h_ref.view(np.uint16)), j
        assert np.array_equal(h, h_ref.astype(np.float64)), j
