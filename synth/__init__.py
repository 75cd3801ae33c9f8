"""Seeded synthetic surface point clouds, normals and right-hand sides.

This module produces the *inputs* that both the CPU oracle and the HIP library
consume. It holds none of the multilevel method's arithmetic (no stencils,
weights, coarsening, transfer operators or solvers); it only samples surfaces
and evaluates right-hand-side functions.

Surfaces (the paper's test problem is a closed smooth surface with a point
cloud and normals, Section 1.1):
  * unit sphere, Fibonacci spiral points, optional tangential jitter;
  * torus R=1, r=1/3, Poisson-disk points by dart throwing (random sequential
    adsorption with a fixed exclusion distance), stopped at exactly N points;
  * star-shaped surface r(w) = 1 + 0.25 g(w)/max|g| with g a random real
    spherical-harmonic expansion of degree <= 6, on Fibonacci points;
  * the same star surface with a 16:1 density contrast (8 Gaussian bumps),
    sampled by variable-radius dart throwing.

Every generator is deterministic for a given `seed_key` (a tuple of ints passed
to numpy's SeedSequence).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


def rng_streams(config_id: int, n_streams: int = 3):
    """Independent generators (points, rhs, mlp) for workload `config_id`."""
    ss = np.random.SeedSequence([2204, 6154, int(config_id)])
    return [np.random.default_rng(s) for s in ss.spawn(n_streams)]


# ----------------------------------------------------------------------------
# Real orthonormal spherical harmonics (fully normalised Legendre recurrence)
# ----------------------------------------------------------------------------
def real_sph_harm_expansion(xyz_unit: np.ndarray, lmax: int, coeffs: np.ndarray) -> np.ndarray:
    """Evaluate sum_{l<=lmax, |m|<=l} a_lm Y_lm at unit vectors.

    `coeffs` has (lmax+1)**2 entries ordered l = 0..lmax, m = -l..l. Y_lm are
    the real orthonormal spherical harmonics (integral of Y_lm^2 over the unit
    sphere is 1), built from the fully normalised associated Legendre
    functions by the standard three-term recurrence in l.
    """
    z = np.clip(xyz_unit[:, 2], -1.0, 1.0)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.arctan2(xyz_unit[:, 1], xyz_unit[:, 0])
    out = np.zeros(xyz_unit.shape[0])
    pmm = np.full_like(z, math.sqrt(1.0 / (4.0 * math.pi)))
    for m in range(lmax + 1):
        if m > 0:
            pmm = -math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * pmm
        cm = np.cos(m * phi)
        sm = np.sin(m * phi)
        p_lm2 = None
        p_lm1 = pmm
        for l in range(m, lmax + 1):
            if l == m:
                p = pmm
            elif l == m + 1:
                p = math.sqrt(2.0 * m + 3.0) * z * pmm
            else:
                a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                a_prev = math.sqrt((4.0 * (l - 1) ** 2 - 1.0) / ((l - 1) ** 2 - m * m))
                p = a * (z * p_lm1 - p_lm2 / a_prev)
            if l > m:
                p_lm2, p_lm1 = p_lm1, p
            base = l * l + l
            if m == 0:
                out += coeffs[base] * p
            else:
                out += coeffs[base + m] * (math.sqrt(2.0) * p * cm)
                out += coeffs[base - m] * (math.sqrt(2.0) * p * sm)
    return out


# ----------------------------------------------------------------------------
# Surfaces
# ----------------------------------------------------------------------------
def fibonacci_sphere(n: int) -> np.ndarray:
    """Fibonacci spiral: z_i = 1-(2i+1)/n, azimuth 2*pi*i/golden."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = 2.0 * math.pi * i / GOLDEN
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def icosahedral_sphere(k: int) -> np.ndarray:
    """Vertices of the icosahedral grid on the unit sphere after k recursive
    subdivisions (each triangle split into four through its edge midpoints,
    projected to the sphere): N = 10 * 4^k + 2 points (k = 5: 10,242)."""
    g = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, g, 0], [1, g, 0], [-1, -g, 0], [1, -g, 0], [0, -1, g], [0, 1, g], [0, -1, -g], [0, 1, -g],
                  [g, 0, -1], [g, 0, 1], [-g, 0, -1], [-g, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4], [11, 10, 2],
                  [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5],
                  [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    for _ in range(k):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e.sort(axis=1)
        ue, inv = np.unique(e, axis=0, return_inverse=True)
        mid = v[ue[:, 0]] + v[ue[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        m = len(v) + inv.reshape(3, -1).T          # midpoint ids of edges (01, 12, 20) of every face
        v = np.concatenate([v, mid])
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        ab, bc, ca = m[:, 0], m[:, 1], m[:, 2]
        f = np.concatenate([np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1), np.stack([ca, bc, c], 1),
                            np.stack([ab, bc, ca], 1)])
    return v


def _sphere_tangent_basis(x: np.ndarray):
    east = np.stack([-x[:, 1], x[:, 0], np.zeros(len(x))], axis=1)
    east /= np.linalg.norm(east, axis=1, keepdims=True)
    north = np.cross(x, east)
    return east, north


def jittered_fibonacci_sphere(n: int, rng: np.random.Generator, jitter: float = 0.1) -> np.ndarray:
    """Fibonacci points moved tangentially by jitter*h*(g1 t1 + g2 t2), h = sqrt(4 pi/n)."""
    x = fibonacci_sphere(n)
    if jitter > 0.0:
        h = math.sqrt(4.0 * math.pi / n)
        t1, t2 = _sphere_tangent_basis(x)
        g = rng.standard_normal((n, 2))
        x = x + jitter * h * (g[:, :1] * t1 + g[:, 1:2] * t2)
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def _dart_throw(candidates: np.ndarray, radius_of, n_target: int, r_max_global: float, k_check: int = 8) -> np.ndarray:
    """Random sequential adsorption in candidate order.

    Candidate c is kept when the kept points p near it satisfy
    |c - p| >= (radius_of(c) + radius_of(p)) / 2 (checked against its k_check
    nearest kept points, and exactly against earlier candidates of its own
    batch). Stops after n_target kept points; returns the kept candidate
    indices in acceptance order.
    """
    kept: list[int] = []
    radii_all = radius_of(candidates)
    batch = max(2048, n_target // 32)
    pos = 0
    while len(kept) < n_target and pos < len(candidates):
        cb = candidates[pos:pos + batch]
        rb = radii_all[pos:pos + batch]
        ok = np.ones(len(cb), dtype=bool)
        if kept:
            karr = np.array(kept, dtype=np.int64)
            tree = cKDTree(candidates[karr])
            kk = min(k_check, len(kept))
            d, idx = tree.query(cb, kk)
            if kk == 1:
                d, idx = d[:, None], idx[:, None]
            ok = np.all(d >= 0.5 * (rb[:, None] + radii_all[karr][idx]), axis=1)
        idx_ok = np.nonzero(ok)[0]
        sub = cb[idx_ok]
        rs = rb[idx_ok]
        pairs = cKDTree(sub).query_pairs(r_max_global, output_type="ndarray") if len(sub) > 1 else np.zeros((0, 2), int)
        if len(pairs):
            a, b = np.minimum(pairs[:, 0], pairs[:, 1]), np.maximum(pairs[:, 0], pairs[:, 1])
            dd = np.linalg.norm(sub[a] - sub[b], axis=1)
            conflict = dd < 0.5 * (rs[a] + rs[b])
            a, b = a[conflict], b[conflict]
        else:
            a = b = np.zeros(0, dtype=np.int64)
        adj: dict[int, list[int]] = {}
        for x, y in zip(a.tolist(), b.tolist()):
            adj.setdefault(x, []).append(y)
        blocked = np.zeros(len(sub), dtype=bool)
        for t in range(len(sub)):
            if blocked[t]:
                continue
            kept.append(pos + int(idx_ok[t]))
            if len(kept) >= n_target:
                break
            for u in adj.get(t, ()):
                blocked[u] = True
        pos += batch
    if len(kept) < n_target:
        raise RuntimeError("dart throwing ran out of candidates")
    return np.array(kept[:n_target], dtype=np.int64)


TORUS_R = 1.0
TORUS_r = 1.0 / 3.0


def torus_point(theta, phi, R=TORUS_R, r=TORUS_r):
    return np.stack([(R + r * np.cos(theta)) * np.cos(phi),
                     (R + r * np.cos(theta)) * np.sin(phi),
                     r * np.sin(theta)], axis=-1)


def torus_poisson_disk(n: int, rng: np.random.Generator, R: float = TORUS_R, r: float = TORUS_r):
    """Exactly n Poisson-disk points on the torus; returns (xyz, normals, theta, phi)."""
    area = 4.0 * math.pi ** 2 * R * r
    # exclusion distance chosen so the jammed RSA count is ~1.5 n
    delta = math.sqrt(0.547 * area * 4.0 / (math.pi * 1.5 * n))
    thetas, phis = [], []
    need = 8 * n
    while sum(len(t) for t in thetas) < need:
        m = need
        th = rng.uniform(0.0, 2.0 * math.pi, m)
        acc = rng.uniform(0.0, 1.0, m) < (R + r * np.cos(th)) / (R + r)
        thetas.append(th[acc])
        phis.append(rng.uniform(0.0, 2.0 * math.pi, m)[acc])
    th = np.concatenate(thetas)[:need]
    ph = np.concatenate(phis)[:need]
    cand = torus_point(th, ph, R, r)
    keep = _dart_throw(cand, lambda c: np.full(len(c), delta), n, delta)
    th, ph = th[keep], ph[keep]
    xyz = torus_point(th, ph, R, r)
    nrm = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), np.sin(th)], axis=1)
    return xyz, nrm, th, ph


@dataclass
class StarSurface:
    coeffs: np.ndarray   # (lmax+1)^2 real SH coefficients
    lmax: int
    gmax: float          # max |g| over a Fibonacci probe
    amp: float = 0.25

    def radius(self, w: np.ndarray) -> np.ndarray:
        return 1.0 + self.amp * real_sph_harm_expansion(w, self.lmax, self.coeffs) / self.gmax

    def points_normals(self, w: np.ndarray):
        """Surface points r(w) w and unit normals (proportional to r w - grad_S r)."""
        w = w / np.linalg.norm(w, axis=1, keepdims=True)
        r = self.radius(w)
        h = 1e-5
        grad = np.zeros_like(w)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            wp = w + e
            wm = w - e
            wp /= np.linalg.norm(wp, axis=1, keepdims=True)
            wm /= np.linalg.norm(wm, axis=1, keepdims=True)
            grad[:, k] = (self.radius(wp) - self.radius(wm)) / (2.0 * h)
        grad_s = grad - np.sum(grad * w, axis=1, keepdims=True) * w
        nrm = r[:, None] * w - grad_s
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        return r[:, None] * w, nrm


def make_star_surface(rng: np.random.Generator, lmax: int = 6, n_probe: int = 1_000_000) -> StarSurface:
    coeffs = rng.standard_normal((lmax + 1) ** 2)
    g = real_sph_harm_expansion(fibonacci_sphere(n_probe), lmax, coeffs)
    return StarSurface(coeffs=coeffs, lmax=lmax, gmax=float(np.max(np.abs(g))))


def star_fibonacci(n: int, rng: np.random.Generator, n_probe: int = 1_000_000):
    surf = make_star_surface(rng, n_probe=n_probe)
    xyz, nrm = surf.points_normals(fibonacci_sphere(n))
    return xyz, nrm, surf


def star_density_points(n: int, rng: np.random.Generator, n_probe: int = 1_000_000,
                        n_bumps: int = 8, contrast: float = 16.0, width: float = 0.3):
    """Star surface with a 16:1 density contrast from Gaussian bumps.

    Density in direction space: rho(w) = 1 + (contrast-1) max_b exp(-|w-w_b|^2/(2 width^2))
    over 8 random unit directions w_b. Directions are drawn uniformly, thinned
    with probability rho/contrast, and selected by variable-radius dart throwing
    with exclusion distance proportional to rho^(-1/2) (spacing varies by
    sqrt(contrast) = 4x); the points are r(w) w on the star surface. Returns
    (xyz, normals, surface, rho at the points).
    """
    surf = make_star_surface(rng, n_probe=n_probe)
    cb = rng.standard_normal((n_bumps, 3))
    cb /= np.linalg.norm(cb, axis=1, keepdims=True)

    def density(w):
        d2 = ((w[:, None, :] - cb[None, :, :]) ** 2).sum(axis=2)
        return 1.0 + (contrast - 1.0) * np.exp(-d2 / (2.0 * width * width)).max(axis=1)

    # estimate the mean density by a uniform sample, then draw ~5n thinned candidates
    probe = rng.standard_normal((200_000, 3))
    probe /= np.linalg.norm(probe, axis=1, keepdims=True)
    mean_rho = float(density(probe).mean())
    m = int(5 * n * contrast / mean_rho) + 1
    w = rng.standard_normal((m, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    rho = density(w)
    w = w[rng.uniform(0.0, 1.0, m) < rho / contrast]
    # jammed RSA count ~ 0.547 (4/pi) int rho/delta0^2 dA = 1.5 n on the unit sphere
    delta0 = math.sqrt(0.547 * 16.0 * mean_rho / (1.5 * n))
    idx = _dart_throw(w, lambda c: delta0 / np.sqrt(density(c)), n, delta0)
    xyz, nrm = surf.points_normals(w[idx])
    return xyz, nrm, surf, density(w[idx])


# ----------------------------------------------------------------------------
# Right-hand sides
# ----------------------------------------------------------------------------
def sh_rhs(xyz: np.ndarray, lmax: int, rng: np.random.Generator) -> np.ndarray:
    """f = sum_{l<=lmax,m} a_lm Y_lm(x/|x|), a_lm ~ N(0,1)."""
    a = rng.standard_normal((lmax + 1) ** 2)
    w = xyz / np.linalg.norm(xyz, axis=1, keepdims=True)
    return real_sph_harm_expansion(w, lmax, a)


def torus_trig_rhs(theta: np.ndarray, phi: np.ndarray, rng: np.random.Generator, pmax: int = 4) -> np.ndarray:
    """f = sum_{|p|,|q|<=pmax} a cos(p th + q ph) + b sin(p th + q ph), minus its discrete mean."""
    f = np.zeros_like(theta)
    for p in range(-pmax, pmax + 1):
        for q in range(-pmax, pmax + 1):
            a, b = rng.standard_normal(2)
            arg = p * theta + q * phi
            f += a * np.cos(arg) + b * np.sin(arg)
    return f - f.mean()


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    xyz: np.ndarray
    normals: np.ndarray
    f: np.ndarray | None
    params: dict


def sphere_workload(n: int = 4096, jitter: float = 0.1, lmax: int = 8, config_id: int = 1) -> Workload:
    """Unit sphere, jittered Fibonacci points, screened Poisson -Delta u + u = f (RBF-FD r^3 + deg 2, k=30)."""
    rp, rf, _ = rng_streams(config_id)
    x = jittered_fibonacci_sphere(n, rp, jitter)
    f = sh_rhs(x, lmax, rf)
    params = dict(disc="rbffd", phs_order=1, poly_degree=2, stencil_size=30, problem="screened",
                  mu=1.0, n_coarse_max=200, n_min=0)
    return Workload(f"sphere{n}", x, x.copy(), f, params)


def sbdf2_workload(n: int = 300_000, dt: float = 0.05, jitter: float = 0.1, lmax: int = 8,
                   config_id: int = 6) -> Workload:
    """Repeated screened solves of SBDF2 time stepping for u_t = Delta u on the
    unit sphere: (I - (2 dt / 3) Delta) u^{n+1} = (4 u^n - u^{n-1}) / 3.
    Jittered Fibonacci points, RBF-FD r^3 + deg 2, k=30; `f` holds u^0, a
    random spherical-harmonic field."""
    rp, rf, _ = rng_streams(config_id)
    x = jittered_fibonacci_sphere(n, rp, jitter)
    u0 = sh_rhs(x, lmax, rf)
    params = dict(disc="rbffd", phs_order=1, poly_degree=2, stencil_size=30, problem="screened",
                  mu=2.0 * dt / 3.0, n_min=250, n_coarse_max=0)
    return Workload(f"sbdf2_{n}", x, x.copy(), u0, params)


def harmonics_workload(n: int = 436_605, jitter: float = 0.1, lmax: int = 8, config_id: int = 7) -> Workload:
    """Shift-invert solves for surface harmonics on the unit sphere: systems
    (D_h - sigma I) v = f with sigma = -1, i.e. the screened form I - mu D_h
    with mu = -1. Jittered Fibonacci points, RBF-FD with l = 5, k = l (PHS
    r^11) and n = (l+1)(l+2) = 42 as in the parameter table; `f` is a random
    spherical-harmonic field (a start vector for the Arnoldi iteration)."""
    rp, rf, _ = rng_streams(config_id)
    x = jittered_fibonacci_sphere(n, rp, jitter)
    f = sh_rhs(x, lmax, rf)
    params = dict(disc="rbffd", phs_order=5, poly_degree=5, stencil_size=42, problem="screened",
                  mu=-1.0, n_min=250, n_coarse_max=0)
    return Workload(f"harmonics{n}", x, x.copy(), f, params)


def geodesic_workload(n: int = 872_773, jitter: float = 0.1, config_id: int = 8) -> Workload:
    """Heat-method geodesics on the unit sphere (exact distance arccos(x . x*)):
    jittered Fibonacci points, LBO by RBF-FD with l = 3, k = 3, n = 20 (the
    parameter table), surface gradient by RBF-FD with l = 2, k = 2, n = 12;
    heat steps dt = 0.01 (3 steps), source node 0. `params` is the Poisson
    problem; the heat handle uses the screened form with mu = dt. `f` is None."""
    rp, _, _ = rng_streams(config_id)
    x = jittered_fibonacci_sphere(n, rp, jitter)
    params = dict(disc="rbffd", phs_order=3, poly_degree=3, stencil_size=20, problem="poisson", mu=0.0,
                  n_min=250, n_coarse_max=0)
    wl = Workload(f"geodesic{n}", x, x.copy(), None, params)
    wl.heat = dict(dt=0.01, steps=3, source=0, grad_phs_order=2, grad_degree=2, grad_stencil=12)
    return wl


def icosahedral_workload(k: int = 5, ell: int = 3, config_id: int = 9) -> Workload:
    """The sphere experiments of the paper's scaling study: icosahedral nodes
    (k subdivisions), the shifted Poisson problem I - Delta (mu = 1) with a
    random right-hand side (standard normal per node), RBF-FD with degree l,
    PHS order k = l and n = (l+1)(l+2) (the parameter table), N_min = 250."""
    _, rf, _ = rng_streams(config_id)
    x = icosahedral_sphere(k)
    f = rf.standard_normal(len(x))
    params = dict(disc="rbffd", phs_order=ell, poly_degree=ell, stencil_size=(ell + 1) * (ell + 2),
                  problem="screened", mu=1.0, n_min=250, n_coarse_max=0)
    return Workload(f"icos{len(x)}_l{ell}", x, x.copy(), f, params)


def torus_workload(n: int = 160_000, config_id: int = 2) -> Workload:
    """Torus, Poisson-disk points, Poisson (bordered) with zero-mean trig f (RBF-FD r^5 + deg 3, k=50)."""
    rp, rf, _ = rng_streams(config_id)
    x, nrm, th, ph = torus_poisson_disk(n, rp)
    f = torus_trig_rhs(th, ph, rf)
    params = dict(disc="rbffd", phs_order=2, poly_degree=3, stencil_size=50, problem="poisson",
                  mu=0.0, n_min=250, n_coarse_max=0)
    return Workload(f"torus{n}", x, nrm, f, params)


def big_sphere_workload(n: int = 1 << 20, lmax: int = 32, config_id: int = 3) -> Workload:
    """Unit sphere, plain Fibonacci points, screened Poisson (GFD deg 2, k=25).

    alpha = 16: with the stencil-radius scale rho of the paper's GFD weight,
    alpha = 4 leaves a 25-point degree-2 stencil almost unweighted, its nearest
    neighbours get weights of the centre's sign and Gauss-Seidel diverges on
    L_h in every ordering; alpha = 16 keeps the stencil compact.
    """
    _, rf, _ = rng_streams(config_id)
    x = fibonacci_sphere(n)
    f = sh_rhs(x, lmax, rf)
    params = dict(disc="gfd", poly_degree=2, stencil_size=25, gfd_alpha=16.0, problem="screened",
                  mu=1.0, n_min=250, n_coarse_max=0)
    return Workload(f"sphere{n}", x, x.copy(), f, params)


def star_workload(n: int = 500_000, config_id: int = 4, n_probe: int = 1_000_000) -> Workload:
    """Star surface on Fibonacci points; batched PHS r^3 + deg 3, k=50 weight systems."""
    rp, _, _ = rng_streams(config_id)
    x, nrm, _ = star_fibonacci(n, rp, n_probe=n_probe)
    params = dict(disc="rbffd", phs_order=1, poly_degree=3, stencil_size=50, problem="screened", mu=1.0)
    return Workload(f"star{n}", x, nrm, None, params)


def star_density_workload(n: int = 500_000, config_id: int = 5, n_probe: int = 1_000_000) -> Workload:
    """Star surface with 16:1 density bumps; screened Poisson, RBF-FD r^3 + deg 2, k=30."""
    rp, rf, _ = rng_streams(config_id)
    x, nrm, _, _ = star_density_points(n, rp, n_probe=n_probe)
    f = sh_rhs(x, 8, rf)
    params = dict(disc="rbffd", phs_order=1, poly_degree=2, stencil_size=30, problem="screened",
                  mu=1.0, n_min=250, n_coarse_max=0)
    return Workload(f"stardens{n}", x, nrm, f, params)
