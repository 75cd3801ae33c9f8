"""Host-side checks of libmgm.so (no GPU): the C ABI loads and exports every
declared symbol, the host setup reproduces the oracle's integer work bit for
bit and its floating-point setup within rounding, and bad inputs map to the
documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import hierarchy, knn
from paper_2204_06154_amd import mgm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "mgm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mgm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = mgm.load()
    names = _declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mgm.EXPORTED)


def test_params_struct_layout_matches_defaults():
    p = mgm.make_params({})
    assert (p.disc, p.phs_order, p.poly_degree, p.stencil_size) == (mgm.RBFFD, 3, 3, 20)
    assert (p.interp_size, p.coarsen_factor, p.n_min, p.nu1, p.nu2) == (3, 4, 250, 1, 1)
    assert p.gfd_alpha == 4.0 and p.mu == 1.0 and p.use_graph == 1
    assert p.device_weights == 1 and p.device_setup == 1 and p.cycle == 0 and p.gs_flow == 1
    assert p.gs_max_width == 96


CASES = [
    ("sphere", lambda: synth.sphere_workload(3000), {"n_coarse_max": 150}),
    ("torus", lambda: synth.torus_workload(6000), {"n_min": 300}),
    # widest rows 50 / 44 / 41 entries: the fine level stays plain, level 1 is patch-blocked
    ("torus_w45", lambda: synth.torus_workload(6000), {"n_min": 300, "gs_max_width": 45}),
    ("gfd", lambda: synth.big_sphere_workload(9001), {"n_min": 200}),
    ("ragged", lambda: synth.sphere_workload(2053), {"n_coarse_max": 100}),
    ("shifted", lambda: synth.harmonics_workload(3000), {}),
    ("icos_l7", lambda: synth.icosahedral_workload(4, 7), {}),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def pair(request):
    _, make, extra = request.param
    wl = make()
    wl.params.update(extra)
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=-1)
    yield wl, H, m
    m.close()


def test_integer_setup_bit_exact(pair):
    wl, H, m = pair
    assert list(m.export("level_sizes")) == [lv.N for lv in H.levels]
    st = m.export("stencils").reshape(len(wl.xyz), -1)
    assert np.array_equal(st, H.stencils)
    for j in range(len(H.levels) - 1):
        lv = H.levels[j]
        assert np.array_equal(m.export("coarse_idx", j), lv.coarse_idx)
        assert np.array_equal(m.export("interp_idx", j).reshape(lv.N, -1), lv.interp_idx)
        assert np.array_equal(m.export("colours", j), lv.colour)
        if lv.patches is not None:
            assert np.array_equal(m.export("patch", j), lv.patches["patch"])
    assert list(m.export("ncolours")) == [lv.ncolours for lv in H.levels[:-1]]
    for j, lv in enumerate(H.levels):
        assert np.array_equal(m.export("l_rowptr", j), lv.pat.indptr)
        assert np.array_equal(m.export("l_cols", j), lv.pat.indices)


# Degree 7 with PHS r^15: the scaled saddle systems reach cond ~2.5e11
# (degree 3: ~6e4, degree 5: ~9e7), so two LU solves may differ by up to
# cond * eps ~ 6e-5 relative; 1e-8 holds with margin (8e-10 measured).
WEIGHT_TOL = {"icos_l7": 1e-8}


def test_float_setup_within_rounding(pair, request):
    """Weights: two pivoted-LU / QR solves of the same local systems differ by
    about cond * eps; the scaled saddle systems have cond up to ~1e4-1e6
    (degree <= 3), so 1e-10 relative to each row's weight magnitude."""
    wl, H, m = pair
    tol = WEIGHT_TOL.get(request.node.callspec.id, 1e-10)
    w = m.export("weights").reshape(H.weights.shape)
    scale = np.abs(H.weights).max(axis=1, keepdims=True)
    assert np.max(np.abs(w - H.weights) / scale) < tol
    for j, lv in enumerate(H.levels):
        v = m.export("l_vals", j)
        L = lv.L
        rows = np.repeat(np.arange(L.shape[0]), np.diff(L.indptr))
        rs = np.maximum.reduceat(np.abs(L.data), L.indptr[:-1])[rows]
        assert np.max(np.abs(v - L.data) / rs) < 10 * tol, j
        if lv.b is not None:
            assert np.max(np.abs(m.export("border", j) - lv.b)) < 1e-10 * np.abs(lv.b).max()
    for j in range(len(H.levels) - 1):
        lv = H.levels[j]
        pw = m.export("interp_w", j).reshape(lv.N, -1)
        Pd = lv.P
        ref = np.zeros_like(pw)
        for t in range(pw.shape[1]):
            ref[:, t] = np.asarray(Pd[np.arange(lv.N), lv.interp_idx[:, t]]).ravel()
        assert np.max(np.abs(pw - ref)) < 1e-12


def test_host_only_handle_rejects_device_calls():
    wl = synth.sphere_workload(600)
    wl.params["n_coarse_max"] = 100
    m = mgm.Mgm(wl.xyz, wl.normals, wl.params, device=-1)
    lib = mgm.load()
    st = lib.mgm_vcycle(m.h, ctypes.c_void_p(8), ctypes.c_void_p(16), None)
    assert st == -1 and b"host-only" in lib.mgm_last_error()
    m.close()


@pytest.mark.parametrize("mutate,status", [
    ("dup", -5), ("nan", -9), ("mu0", -1), ("muinf", -1), ("tiny", -1), ("onelevel", -1), ("badstencil", -1),
    ("collinear", -4), ("gsflow3", -1), ("phs0", -1),
])
def test_failure_injection(mutate, status):
    wl = synth.sphere_workload(800)
    wl.params["n_coarse_max"] = 100
    x, nrm, p = wl.xyz.copy(), wl.normals.copy(), dict(wl.params)
    if mutate == "dup":
        x[5] = x[600]
    elif mutate == "nan":
        x[3, 1] = np.nan
    elif mutate == "mu0":
        p["mu"] = 0.0
    elif mutate == "muinf":
        p["mu"] = -np.inf
    elif mutate == "tiny":
        x, nrm = x[:10], nrm[:10]
    elif mutate == "onelevel":
        # N < 4 N_min: the level count of Alg. 2 is 1, no level to smooth
        p.pop("n_coarse_max")
        p["n_min"] = 250
        x, nrm = x[:600], nrm[:600]
    elif mutate == "gsflow3":
        p["gs_flow"] = 3
    elif mutate == "phs0":
        p["phs_order"] = 0  # r^1: its Laplacian is infinite at the stencil centre
    elif mutate == "badstencil":
        p["stencil_size"] = 3   # fewer than the 6 degree-2 monomials
    elif mutate == "collinear":
        # all points on one great circle: every tangent stencil is collinear
        t = np.linspace(0, 2 * np.pi, 800, endpoint=False)
        x = np.stack([np.cos(t), np.sin(t), np.zeros_like(t)], axis=1)
        nrm = x.copy()
    with pytest.raises(mgm.MgmError) as ei:
        mgm.Mgm(x, nrm, p, device=-1)
    assert ei.value.status == status


def test_library_stencils_bit_exact():
    from oracle import knn
    x = synth.torus_workload(5000).xyz
    for k in (2, 3, 25, 50):
        assert np.array_equal(mgm.stencils(x, k), knn.stencils(x, k)), k


def test_surface_gradient_weights_match_oracle():
    """Library surface-gradient operator (host-only handle) against the
    oracle's: stencils bit for bit, weights to the rounding of two LU solves."""
    from oracle import geodesic
    wl = synth.geodesic_workload(3000)
    m = mgm.Mgm(wl.xyz, wl.normals, dict(wl.params, device_weights=0), device=-1)
    try:
        with pytest.raises(mgm.MgmError):
            m.surface_ops_setup(0, 2, 12)          # needs r^3 or smoother
        m.surface_ops_setup(2, 2, 12)
        n = len(wl.xyz)
        sten = m.export("grad_stencils").reshape(n, 12)
        assert np.array_equal(sten, knn.stencils(wl.xyz, 12))
        W = m.export("grad_weights").reshape(n, 12, 3)
        ref = geodesic.surface_gradient_operator(wl.xyz, wl.normals, sten, 2, 2)
        scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
        assert np.max(np.abs(W - ref) / scale) < 1e-10
    finally:
        m.close()
