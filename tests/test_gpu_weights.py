"""Batched device RBF-FD weight solves (eq. rbf_fd_lap) against the oracle.

Parity: the device solves the same saddle systems by Gauss-Jordan with
partial pivoting, the oracle by LAPACK's LU; both are accurate to ~cond*eps
of the scaled system, so weights agree to 1e-10 of each row's magnitude.
Independent pin at any size: polynomial reproduction sum_j c_ij p(xh_j) =
Lap p(0) for every monomial of degree <= l (the saddle system's constraint
rows), at 1e-10 relative (the acceptance criterion of the batched workload).
"""
import numpy as np
import pytest

import synth
from oracle import discretize, knn
from paper_2204_06154_amd import mgm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _poly_repro_error(xyz, nrm, sten, c, deg, centres=None):
    """Worst scaled |sum_j c_ij p(xh_j) - Lap p(0)| over monomials; row i of
    sten/c is the stencil of point centres[i] (default: point i)."""
    if centres is None:
        centres = np.arange(len(sten))
    d = xyz[sten] - xyz[centres][:, None, :]
    t1, t2 = discretize.tangent_frames(nrm[centres])
    xh = np.stack([np.einsum("inc,ic->in", d, t1), np.einsum("inc,ic->in", d, t2)], axis=2)
    s = np.sqrt((xh ** 2).sum(axis=2)).max(axis=1)
    worst = 0.0
    for a, b in discretize.monomial_exponents(deg):
        val = (c * xh[..., 0] ** a * xh[..., 1] ** b).sum(axis=1)
        exact = 2.0 if (a, b) in ((2, 0), (0, 2)) else 0.0
        scale = np.abs(c).sum(axis=1) * s ** (a + b)
        worst = max(worst, float(np.max(np.abs(val - exact) / scale)))
    return worst


@pytest.mark.parametrize("surface,phs,deg,k", [("sphere", 1, 2, 30), ("torus", 2, 3, 50), ("star", 1, 3, 50),
                                                ("star", 2, 2, 20), ("torus", 1, 0, 7), ("sphere", 5, 5, 42)])
def test_batched_weights_match_oracle(surface, phs, deg, k):
    if surface == "sphere":
        wl = synth.sphere_workload(3000)
    elif surface == "torus":
        wl = synth.torus_workload(3000)
    else:
        wl = synth.star_workload(3001, n_probe=20000)
    sten = knn.stencils(wl.xyz, k)
    lib_sten = mgm.stencils(wl.xyz, k)
    assert np.array_equal(sten, lib_sten)
    d_x = torch.tensor(wl.xyz, device="cuda")
    d_n = torch.tensor(wl.normals, device="cuda")
    d_s = torch.tensor(lib_sten, device="cuda")
    c = mgm.batched_weights(d_x, d_n, d_s, phs, deg).cpu().numpy()
    ref = discretize.rbffd_weights(discretize.project_stencils(wl.xyz, wl.normals, sten), phs, deg)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.max(np.abs(c - ref) / scale) < 1e-10
    assert _poly_repro_error(wl.xyz, wl.normals, sten, c, deg) < 1e-10


def test_batched_weights_full_size_sampled():
    """The 500,000-system star-surface workload (n=50, r^3 + degree 3): sampled
    rows against the oracle one by one, and polynomial reproduction on all."""
    wl = synth.star_workload(500_000)
    sten = mgm.stencils(wl.xyz, 50)
    d_x = torch.tensor(wl.xyz, device="cuda")
    d_n = torch.tensor(wl.normals, device="cuda")
    d_s = torch.tensor(sten, device="cuda")
    c = mgm.batched_weights(d_x, d_n, d_s, 1, 3).cpu().numpy()
    rows = np.random.default_rng(0).choice(len(wl.xyz), 2000, replace=False)
    sten_o, _ = knn.knn(wl.xyz[rows], wl.xyz, 50)
    assert np.array_equal(sten_o, sten[rows])
    d = wl.xyz[sten_o] - wl.xyz[rows][:, None, :]
    t1, t2 = discretize.tangent_frames(wl.normals[rows])
    xh = np.stack([np.einsum("inc,ic->in", d, t1), np.einsum("inc,ic->in", d, t2)], axis=2)
    ref = discretize.rbffd_weights(xh, 1, 3)
    assert np.max(np.abs(c[rows] - ref) / np.abs(ref).max(axis=1, keepdims=True)) < 1e-10
    for s0 in range(0, len(wl.xyz), 100_000):
        sl = slice(s0, s0 + 100_000)
        assert _poly_repro_error(wl.xyz, wl.normals, sten[sl], c[sl], 3, np.arange(len(wl.xyz))[sl]) < 1e-10


def test_singular_stencil_reported():
    t = np.linspace(0, 2 * np.pi, 300, endpoint=False)
    x = np.stack([np.cos(t), np.sin(t), np.zeros_like(t)], axis=1)   # collinear stencils
    sten = mgm.stencils(x, 20)
    with pytest.raises(mgm.MgmError) as ei:
        mgm.batched_weights(torch.tensor(x, device="cuda"), torch.tensor(x, device="cuda"),
                            torch.tensor(sten, device="cuda"), 1, 2)
    assert ei.value.status == -4


def test_setup_with_device_weights_matches_host_weights():
    wl = synth.torus_workload(4000)
    p_dev = dict(wl.params, n_min=200, device_weights=1)
    p_host = dict(wl.params, n_min=200, device_weights=0)
    a = mgm.Mgm(wl.xyz, wl.normals, p_dev, device=0)
    b = mgm.Mgm(wl.xyz, wl.normals, p_host, device=0)
    wa, wb = a.export("weights"), b.export("weights")
    assert np.max(np.abs(wa - wb)) < 1e-10 * np.abs(wb).max()
    for j in range(len(a.export("level_sizes")) - 1):
        assert np.array_equal(a.export("colours", j), b.export("colours", j))
    a.close()
    b.close()


@pytest.mark.parametrize("noalloc", [False, True])
def test_empty_batch_and_size_checks(noalloc):
    """An empty batch returns at once (null stencil and weight pointers
    allowed) but still checks its sizes; a system above 64 unknowns is an
    argument error."""
    wl = synth.sphere_workload(500)
    d_x = torch.tensor(wl.xyz, device="cuda")
    d_n = torch.tensor(wl.normals, device="cuda")
    d_s = torch.empty((0, 30), dtype=torch.int32, device="cuda")
    w = mgm.batched_weights(d_x, d_n, d_s, 1, 2, noalloc=noalloc,
                            d_weights=torch.empty((0, 30), dtype=torch.float64, device="cuda"))
    assert tuple(w.shape) == (0, 30)
    with pytest.raises(mgm.MgmError) as ei:   # 60 + 28 unknowns (degree 6) > 64
        mgm.batched_weights(d_x, d_n, torch.empty((0, 60), dtype=torch.int32, device="cuda"), 1, 6, noalloc=noalloc,
                            d_weights=torch.empty((0, 60), dtype=torch.float64, device="cuda"))
    assert ei.value.status == -1


@pytest.mark.parametrize("surface,phs,deg,k", [("sphere", 1, 2, 30), ("torus", 2, 3, 50), ("star", 1, 3, 50),
                                                ("star", 2, 2, 20), ("torus", 1, 0, 7), ("sphere", 3, 4, 45)])
def test_mixed_precision_weights_match_oracle(surface, phs, deg, k):
    """FP32 elimination on the matrix cores with FP64 refinement: the same
    bar as the FP64 elimination (1e-10 of each row's magnitude against the
    oracle's LAPACK solve, polynomial reproduction to 1e-10)."""
    if surface == "sphere":
        wl = synth.sphere_workload(3000)
    elif surface == "torus":
        wl = synth.torus_workload(3000)
    else:
        wl = synth.star_workload(3001, n_probe=20000)
    sten = knn.stencils(wl.xyz, k)
    d_x = torch.tensor(wl.xyz, device="cuda")
    d_n = torch.tensor(wl.normals, device="cuda")
    d_s = torch.tensor(sten.astype(np.int32), device="cuda")
    c = mgm.batched_weights(d_x, d_n, d_s, phs, deg, mixed=True).cpu().numpy()
    ref = discretize.rbffd_weights(discretize.project_stencils(wl.xyz, wl.normals, sten), phs, deg)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    err = np.max(np.abs(c - ref) / scale)
    print(f"[gpu-weights-mixed] {surface} phs {phs} deg {deg} k {k}: max rel err {err:.2e}", flush=True)
    assert err < 1e-10
    assert _poly_repro_error(wl.xyz, wl.normals, sten, c, deg) < 1e-10


def test_mixed_precision_weights_need_degree_at_most_four():
    wl = synth.sphere_workload(500)
    d_x = torch.tensor(wl.xyz, device="cuda")
    d_n = torch.tensor(wl.normals, device="cuda")
    d_s = torch.tensor(knn.stencils(wl.xyz, 30).astype(np.int32), device="cuda")
    with pytest.raises(mgm.MgmError) as ei:
        mgm.batched_weights(d_x, d_n, d_s, 1, 5, mixed=True)
    assert ei.value.status == -1
