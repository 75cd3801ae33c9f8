"""Pins of the oracle's setup steps against brute force, closed forms and identities.

Each test fixes a step of the CPU oracle to something other than itself, so
that a dropped term, a wrong sign or index, or a transposed operand fails.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import coarsen, colouring, discretize, galerkin, hierarchy, knn, transfer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- kNN (Sec. 2)
def _knn_brute(q, d, k):
    D2 = knn.sq_dist(q[:, None, :], d[None, :, :])
    out = []
    for i in range(len(q)):
        order = np.lexsort((np.arange(len(d)), D2[i]))
        out.append(order[:k])
    return np.array(out)


def test_knn_matches_bruteforce_random():
    rng = np.random.default_rng(0)
    x = synth.jittered_fibonacci_sphere(700, rng, 0.3)
    idx, _ = knn.knn(x, x, 25)
    assert np.array_equal(idx, _knn_brute(x, x, 25))


def test_knn_ties_broken_by_index():
    # integer lattice: many exactly equal distances
    g = np.arange(7, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    pts = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    perm = np.random.default_rng(1).permutation(len(pts))
    pts = pts[perm]
    idx, _ = knn.knn(pts, pts, 13)
    assert np.array_equal(idx, _knn_brute(pts, pts, 13))
    assert np.all(idx[:, 0] == np.arange(len(pts)))


def test_knn_coarse_queries():
    rng = np.random.default_rng(2)
    x = synth.jittered_fibonacci_sphere(600, rng, 0.3)
    y = x[rng.choice(600, 150, replace=False)]
    idx, _ = knn.knn(x, y, 3)
    assert np.array_equal(idx, _knn_brute(x, y, 3))


def test_duplicate_points_rejected():
    x = synth.fibonacci_sphere(200)
    x[17] = x[90]
    with pytest.raises(knn.DuplicatePointsError):
        knn.stencils(x, 10)


# ------------------------------------------------------- weights (Sec. 2.2-2.3)
def _flat_cross():
    h = 0.1
    return np.array([[0, 0], [h, 0], [-h, 0], [0, h], [0, -h], [h, h]], dtype=np.float64), h


def test_rbffd_reduces_to_five_point_laplacian():
    # n = L = 6 with degree 2: the polynomial constraints fix the weights, which
    # are the quadratic-interpolation weights: the textbook 5-point stencil.
    xh, h = _flat_cross()
    c = discretize.rbffd_weights(xh[None], phs_order=1, deg=2)[0]
    ref = np.array([-4, 1, 1, 1, 1, 0]) / h ** 2
    assert np.allclose(c, ref, rtol=0, atol=1e-9 / h ** 2)


def test_gfd_reduces_to_five_point_laplacian():
    xh, h = _flat_cross()
    sten = np.zeros((1, 6), dtype=np.int64)
    c = discretize.gfd_weights(xh[None], sten, deg=2, alpha=4.0)[0]
    ref = np.array([-4, 1, 1, 1, 1, 0]) / h ** 2
    assert np.allclose(c, ref, rtol=0, atol=1e-9 / h ** 2)


@pytest.mark.parametrize("disc,phs,deg,n", [("rbffd", 1, 2, 30), ("rbffd", 2, 3, 50), ("rbffd", 1, 3, 50),
                                            ("gfd", 0, 2, 25)])
def test_polynomial_reproduction_and_row_sums(disc, phs, deg, n):
    """sum_j c_ij p(xh_j) = Lap p(0) for every monomial of degree <= l (eqs. rbf_fd_lap, wls_fd_lap)."""
    wl = synth.star_workload(3000, n_probe=20000)
    sten = knn.stencils(wl.xyz, n)
    xh = discretize.project_stencils(wl.xyz, wl.normals, sten)
    params = dict(disc=disc, phs_order=phs, poly_degree=deg, gfd_alpha=4.0)
    c = discretize.lbo_weights(wl.xyz, wl.normals, sten, params)
    s = np.sqrt((xh ** 2).sum(axis=2)).max(axis=1)
    for a, b in discretize.monomial_exponents(deg):
        # unscaled monomials in tangent coordinates; Lap(x^a y^b)(0) = 2 for x^2, y^2
        val = (c * xh[..., 0] ** a * xh[..., 1] ** b).sum(axis=1)
        exact = 2.0 if (a, b) in ((2, 0), (0, 2)) else 0.0
        scale = np.abs(c).sum(axis=1) * s ** (a + b)
        assert np.max(np.abs(val - exact) / scale) < 1e-10, (a, b)
    assert np.max(np.abs(c.sum(axis=1)) / np.abs(c).sum(axis=1)) < 1e-12


def _y54(x):
    return x[:, 2] * (x[:, 0] ** 4 - 6 * x[:, 0] ** 2 * x[:, 1] ** 2 + x[:, 1] ** 4)


def _lbo_error(n, disc, phs, deg, k):
    x = synth.fibonacci_sphere(n)
    sten = knn.stencils(x, k)
    c = discretize.lbo_weights(x, x, sten, dict(disc=disc, phs_order=phs, poly_degree=deg, gfd_alpha=4.0))
    u = _y54(x)
    lap = (c * u[sten]).sum(axis=1)
    return np.max(np.abs(lap - (-30.0) * u)) / np.max(np.abs(30.0 * u))


@pytest.mark.parametrize("disc,phs,deg,k,order", [("rbffd", 1, 2, 30, 1.0), ("rbffd", 2, 3, 50, 1.8),
                                                   ("gfd", 0, 2, 25, 1.0)])
def test_lbo_spherical_harmonic_convergence(disc, phs, deg, k, order):
    """D_h Y_5^4 -> -30 Y_5^4 on the unit sphere, error falling with N (eigenvalue from golden)."""
    (lval, eig), = _golden("sphere_y54.txt")
    assert int(eig) == -int(lval) * (int(lval) + 1)
    e1 = _lbo_error(4096, disc, phs, deg, k)
    e2 = _lbo_error(16384, disc, phs, deg, k)
    rate = math.log(e1 / e2) / math.log(2.0)    # h halves when N quadruples
    assert e2 < 0.05 and rate > order, (e1, e2, rate)


# ------------------------------------------------------------- WSE (Sec. 4.1)
@pytest.mark.parametrize("n,seed", [(400, 0), (1200, 1)])
def test_wse_heap_matches_bruteforce(n, seed):
    x = synth.jittered_fibonacci_sphere(n, np.random.default_rng(seed), 0.4)
    a = coarsen.wse(x)
    b = coarsen.wse_bruteforce(x)
    assert np.array_equal(a, b)
    assert len(a) == n // 4 and np.all(np.diff(a) > 0)


def test_wse_improves_separation_over_random_subset():
    x = synth.jittered_fibonacci_sphere(4000, np.random.default_rng(3), 0.4)
    keep = coarsen.wse(x)
    rnd = np.random.default_rng(4).choice(len(x), len(keep), replace=False)

    def sep(pts):
        _, d2 = knn.knn(pts, pts, 2)
        return np.sqrt(d2[:, 1].min())
    assert sep(x[keep]) > 2.0 * sep(x[rnd])
    # quasi-uniform: min separation close to the mean spacing of a 1000-point cloud
    assert sep(x[keep]) > 0.5 * math.sqrt(4 * math.pi / len(keep))


@pytest.mark.parametrize("n1", [4096, 10000, 160000, 1 << 20, 500000, 300, 999, 1000, 1001, 64000, 64001])
def test_level_count_formula(n1):
    """p = floor(log(N_1/N_min)/log 4) + 1 and N_min <= N_p < 4 N_min (Alg. 2)."""
    sizes = coarsen.level_sizes(n1, 250)
    p_formula = math.floor(math.log(n1 / 250) / math.log(4) + 1e-12) + 1
    assert len(sizes) == p_formula
    assert 250 <= sizes[-1] < 1000
    for j, s in enumerate(sizes):
        assert s == n1 // 4 ** j


def test_level_sizes_coarse_max_rule():
    assert coarsen.level_sizes(4096, 0, 200) == [4096, 1024, 256, 64]


def test_table1_defaults():
    g = {k: int(v) for k, v in _golden("table1_parameters.txt")}
    d = hierarchy.DEFAULTS
    assert d["n_min"] == g["n_min"] and d["interp_size"] == g["interp_size"]
    assert d["coarsen_factor"] == g["coarsen_factor"]
    for l in (3, 5, 7):
        assert (l + 1) * (l + 2) == g[f"stencil_l{l}"]


# ---------------------------------------------------- interpolation (Sec. 3)
def test_interpolation_reproduces_constants_and_injects():
    x = synth.jittered_fibonacci_sphere(2000, np.random.default_rng(5), 0.3)
    keep = coarsen.wse(x)
    P, idx, inj = transfer.interpolation(x, x[keep], 3)
    assert np.max(np.abs(P @ np.ones(P.shape[1]) - 1.0)) < 1e-14
    # nested: every survivor row is exactly the unit row of itself
    assert np.all(inj[keep])
    Pd = P[keep].toarray()
    assert np.array_equal(Pd, np.eye(len(keep)))
    nnz = np.diff(P.indptr)
    assert set(np.unique(nnz[~inj])) <= {3}


def test_interpolation_weights_equal_interpolant_evaluation():
    """d = weights from eq. rbf_fd_interp; evaluating the interpolant built from data
    (the transposed system) at x_i must give sum_j d_ij u_j for any data u."""
    rng = np.random.default_rng(6)
    x = synth.jittered_fibonacci_sphere(800, rng, 0.3)
    keep = coarsen.wse(x)
    y = x[keep]
    P, idx, inj = transfer.interpolation(x, y, 3)
    u = rng.standard_normal(len(y))
    Pu = P @ u
    for i in np.nonzero(~inj)[0][:50]:
        yy = y[idx[i]]
        A = np.linalg.norm(yy[:, None, :] - yy[None, :, :], axis=2)
        M = np.block([[A, np.ones((3, 1))], [np.ones((1, 3)), np.zeros((1, 1))]])
        coef = np.linalg.solve(M, np.concatenate([u[idx[i]], [0.0]]))
        s = np.linalg.norm(x[i] - yy, axis=1) @ coef[:3] + coef[3]
        assert abs(s - Pu[i]) < 1e-12 * (1 + abs(s))


# ----------------------------------------------------- Galerkin (Sec. 4.2, 4.4)
def test_galerkin_dense_and_constant_identity():
    wl = synth.torus_workload(3000)
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    for j in range(len(H.levels) - 1):
        lv, nx = H.levels[j], H.levels[j + 1]
        dense = lv.P.toarray().T @ lv.L.toarray() @ lv.P.toarray()
        assert np.max(np.abs(nx.L.toarray() - dense)) < 1e-12 * np.abs(dense).max()
        # Poisson: L 1 = 0 (zero row sums) and P 1 = 1 give L_H 1 = 0
        one = np.ones(nx.N)
        assert np.max(np.abs(nx.L @ one)) < 1e-10 * abs(nx.L).max()
        # border b_H = P^T b_h, and sum(b_H) = N_h because rows of P sum to 1
        assert np.allclose(nx.b, lv.P.T @ lv.b)
        assert abs(nx.b.sum() - lv.b.sum()) < 1e-9 * lv.b.sum()
        # structural pattern contains the numeric pattern
        assert (abs(nx.L) > 0).astype(int).multiply(1 - nx.pat.toarray()).sum() == 0


# ----------------------------------------------------- colouring / hashing
def test_splitmix64_published_values():
    rows = _golden("splitmix64.txt")
    args = np.array([int(a, 16) for a, _ in rows], dtype=np.uint64)
    vals = [int(v, 16) for _, v in rows]
    assert [int(v) for v in colouring.splitmix64(args)] == vals


def _jp_sequential(G):
    """Jones-Plassmann written as plain loops (for tiny graphs)."""
    N = G.shape[0]
    prio = colouring.priorities(G)
    adj = [G.indices[G.indptr[i]:G.indptr[i + 1]].tolist() for i in range(N)]
    colour = [-1] * N
    while -1 in colour:
        sel = [v for v in range(N) if colour[v] < 0 and all(colour[u] >= 0 or prio[u] < prio[v] for u in adj[v])]
        new = {}
        for v in sel:
            used = {colour[u] for u in adj[v] if colour[u] >= 0}
            c = 0
            while c in used:
                c += 1
            new[v] = c
        for v, c in new.items():
            colour[v] = c
    return np.array(colour)


def test_colouring_matches_plain_loops_and_is_valid():
    wl = synth.sphere_workload(1500)
    wl.params["n_coarse_max"] = 100
    wl.params["gs_block"] = 0
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    for lv in H.levels[:-1]:
        assert colouring.is_valid_colouring(lv.pat, lv.colour)
        G = colouring.symmetric_graph(lv.pat)
        assert np.array_equal(lv.colour, _jp_sequential(G))


def _rcb_plain(x, ids, block, out, nxt):
    """Recursive coordinate bisection written as plain recursion (tiny sets)."""
    if len(ids) <= block:
        for i in ids:
            out[i] = nxt
        return nxt + 1
    ext = [max(x[i, a] for i in ids) - min(x[i, a] for i in ids) for a in range(3)]
    axis = ext.index(max(ext))
    ids = sorted(ids, key=lambda i: (x[i, axis], i))
    cut = (-(-len(ids) // block) // 2) * block
    nxt = _rcb_plain(x, ids[:cut], block, out, nxt)
    return _rcb_plain(x, ids[cut:], block, out, nxt)


def _dsatur_plain(G):
    """DSATUR written as a plain scan over all nodes at every step (tiny graphs)."""
    N = G.shape[0]
    adj = [G.indices[G.indptr[i]:G.indptr[i + 1]].tolist() for i in range(N)]
    colour = [-1] * N
    for _ in range(N):
        best = None
        for v in range(N):
            if colour[v] >= 0:
                continue
            key = (len({colour[u] for u in adj[v] if colour[u] >= 0}), len(adj[v]), -v)
            if best is None or key > best[0]:
                best = (key, v)
        v = best[1]
        used = {colour[u] for u in adj[v] if colour[u] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[v] = c
    return np.array(colour)


def _rlf_plain(G):
    """Recursive largest first with every count recomputed from the sets at
    every pick (tiny graphs)."""
    N = G.shape[0]
    adj = [set(G.indices[G.indptr[i]:G.indptr[i + 1]].tolist()) for i in range(N)]
    colour = [-1] * N
    uncol = set(range(N))
    c = 0
    while uncol:
        elig, excl = set(uncol), set()
        v = max(elig, key=lambda x: (len(adj[x] & uncol), -x))
        while True:
            colour[v] = c
            uncol.discard(v)
            elig.discard(v)
            moved = adj[v] & elig
            elig -= moved
            excl |= moved
            if not elig:
                break
            v = max(elig, key=lambda x: (len(adj[x] & excl), -len(adj[x] & elig), -x))
        c += 1
    return np.array(colour)


def test_rlf_known_cases():
    def graph(n, edges):
        e = np.array(edges)
        return colouring.symmetric_graph(sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n)).tocsr())
    # path 0-1-2-3: the class of node 1 (largest degree, smaller index) takes 3 as well
    assert colouring.rlf_colouring(graph(4, [(0, 1), (1, 2), (2, 3)])).tolist() == [1, 0, 1, 0]
    # star with centre 4: the first class is the centre alone, then all leaves
    assert colouring.rlf_colouring(graph(5, [(4, k) for k in range(4)])).tolist() == [1, 1, 1, 1, 0]
    # odd cycle: three colours; complete graph K_6: six
    assert colouring.rlf_colouring(graph(9, [(k, (k + 1) % 9) for k in range(9)])).max() == 2
    assert sorted(colouring.rlf_colouring(colouring.symmetric_graph(sp.csr_matrix(np.ones((6, 6)))))) == list(range(6))
    # random graphs: valid, and the same as the plain recount
    rng = np.random.default_rng(11)
    for n in (30, 60):
        A = sp.random(n, n, density=0.12, random_state=rng, format="csr")
        G = colouring.symmetric_graph(A)
        c = colouring.rlf_colouring(G)
        assert colouring.is_valid_colouring(A, c)
        assert np.array_equal(c, _rlf_plain(G))


def test_rcb_patches_on_a_grid_are_rectangles():
    """A 32 x 16 grid in the plane cut into patches of 64 points: the longer
    axis is halved until 8 x 8 squares remain, numbered left half first."""
    gx, gy = np.meshgrid(np.arange(32.0), np.arange(16.0), indexing="ij")
    x = np.stack([gx.ravel(), gy.ravel(), np.zeros(gx.size)], axis=1)
    p = colouring.rcb_patches(x, 64)
    assert p.max() + 1 == 8
    for k in range(8):
        sel = x[p == k]
        assert len(sel) == 64
        assert np.ptp(sel[:, 0]) == 7 and np.ptp(sel[:, 1]) == 7
    # depth-first numbering: the first four patches cover x < 16
    assert np.all(x[p < 4, 0] < 16) and np.all(x[p >= 4, 0] >= 16)


def test_dsatur_known_cases():
    rng = np.random.default_rng(5)
    # bipartite graphs (a random tree, an even cycle, a grid) take exactly two colours (Brelaz 1979)
    n = 60
    parent = [int(rng.integers(i)) for i in range(1, n)]
    T = sp.coo_matrix((np.ones(n - 1), (np.arange(1, n), parent)), shape=(n, n)).tocsr()
    cyc = sp.coo_matrix((np.ones(20), (np.arange(20), (np.arange(20) + 1) % 20)), shape=(20, 20)).tocsr()
    g = np.arange(48).reshape(6, 8)
    rows = np.concatenate([g[:, :-1].ravel(), g[:-1, :].ravel()])
    cols = np.concatenate([g[:, 1:].ravel(), g[1:, :].ravel()])
    grid = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(48, 48)).tocsr()
    for A in (T, cyc, grid):
        G = colouring.symmetric_graph(A)
        c = colouring.dsatur_colouring(G)
        assert c.max() == 1 and colouring.is_valid_colouring(A, c)
    # odd cycle: three colours; complete graph K_7: seven
    odd = sp.coo_matrix((np.ones(21), (np.arange(21), (np.arange(21) + 1) % 21)), shape=(21, 21)).tocsr()
    assert colouring.dsatur_colouring(colouring.symmetric_graph(odd)).max() == 2
    K = sp.csr_matrix(np.ones((7, 7)))
    assert sorted(colouring.dsatur_colouring(colouring.symmetric_graph(K))) == list(range(7))


def test_patch_colouring_pins():
    wl = synth.sphere_workload(3000)
    wl.params["n_coarse_max"] = 150
    wl.params["gs_block"] = 64
    H = hierarchy.build(wl.xyz, wl.normals, wl.params)
    for lv in H.levels[:-1]:
        assert lv.patches is not None
        # composite colours are a valid colouring (rows of one colour never couple)
        assert colouring.is_valid_colouring(lv.pat, lv.colour)
        # patches by recursive coordinate bisection (plain recursion)
        x = lv.xyz
        patch = np.empty(len(x), dtype=np.int64)
        _rcb_plain(x, list(range(len(x))), 64, patch, 0)
        assert np.array_equal(patch, lv.patches["patch"])
        sizes = np.bincount(patch)
        assert np.all(sizes[:-1] == 64) and 0 < sizes[-1] <= 64
        # patch colours follow recursive largest first, local colours DSATUR
        G = colouring.symmetric_graph(lv.pat)
        rows = np.repeat(np.arange(G.shape[0]), np.diff(G.indptr))
        cross = patch[rows] != patch[G.indices]
        npatch = patch.max() + 1
        PG = sp.csr_matrix((np.ones(cross.sum()), (patch[rows][cross], patch[G.indices][cross])),
                           shape=(npatch, npatch))
        PG.sum_duplicates()
        PG.sort_indices()
        assert np.array_equal(lv.patches["pcolour"], _rlf_plain(PG))
        GI = sp.csr_matrix((np.ones((~cross).sum()), (rows[~cross], G.indices[~cross])), shape=G.shape)
        GI.sort_indices()
        if G.shape[0] <= 800:  # the plain scan is quadratic
            assert np.array_equal(lv.patches["lcolour"], _dsatur_plain(GI))
        else:  # per patch: DSATUR never looks across the patch boundary
            for k in range(0, npatch, max(1, npatch // 6)):
                ids = np.nonzero(patch == k)[0]
                assert np.array_equal(lv.patches["lcolour"][ids], _dsatur_plain(GI[ids][:, ids]))
        # the GS order is (patch colour, local colour): check the relabelling keeps it
        comp = lv.patches["pcolour"][patch] * (lv.patches["lcolour"].max() + 1) + lv.patches["lcolour"]
        assert np.all(np.diff(comp[np.argsort(lv.colour, kind="stable")]) >= 0)


def test_priorities_largest_degree_first():
    G = sp.csr_matrix(np.array([[0, 1, 1, 1], [1, 0, 0, 0], [1, 0, 0, 1], [1, 0, 1, 0]]))
    p = colouring.priorities(G)
    assert p[0] == 3  # degree 3 beats everyone
    c = colouring.jp_colouring(G)
    assert c[0] == 0 and len(set(c[[0, 2, 3]])) == 3
