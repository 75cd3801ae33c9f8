"""Learned per-node Chebyshev smoother (not in the paper; our reading).

The paper smooths with Gauss-Seidel (Sec. 4.3). This extension replaces the
fine-level smoother by s damped-Jacobi (Richardson) steps with per-node step
weights predicted by a small MLP from the local stencil:

  features_i  = [ xh_j / rho_i (2 values), c_ij / |c_ii| (1 value) ] over the
                stencil of node i in distance order (3n values; n = 30 -> 90),
                xh the tangent-plane coordinates of Sec. 2.1, c the LBO
                weights of Sec. 2.2, rho_i = max_j |xh_j|;
  MLP         = 3n -> 64 -> 64 -> s, ReLU, FP32 (FP64 here);
  omega_{q,i} = omega_q (1 + 0.5 tanh(o_{q,i})),  omega_q = 1/theta_q,
  theta_q     = (b+a)/2 + (b-a)/2 cos((2q-1) pi / (2s)),  q = 1..s,
                the Chebyshev roots on [a, b] = [lam/4, 1.1 lam], lam a
                20-step power-iteration estimate of rho(D^-1 L);
  smoother    = for q = 1..s:  e <- e + omega_q * D^-1 (r - L e).

With a zero last layer the step weights are 1/theta_q and the error
propagation polynomial is the scaled Chebyshev polynomial on [a, b].

Training (homogeneous problem L e = 0): error snapshots e_t are taken right
after the coarse-grid correction of MGM iterations started from random
errors; the loss is mean_t |L S_w e_t|^2 / |L e_t|^2. Backward (adjoint of the
smoother): g_s = 2 L^T L e_s / |L e_0|^2; for q = s..1:
dLoss/domega_q = -g_q * z_q with z_q = D^-1 L e_{q-1}, and
g_{q-1} = g_q - L^T D^-1 (omega_q * g_q). Adam (Kingma & Ba 2015).

Random numbers: the power-iteration start and the weight initialisation use
SplitMix64 as a counter-based generator, u(k) = (splitmix64(k) >> 11) 2^-53.

Per-level smoothing (also our reading): a coarse level j gets a smoother of
the same form with its own MLP, lam_j and step weights. Coarse points are
fine points, so they carry normals; the features of coarse node i are its n
nearest level-j points (n capped at N_j; centre first) in the tangent plane,
scaled by the stencil radius, and the entries of the Galerkin operator L_j
at those points over |L_j(i,i)| (0 where L_j has no entry). Level j trains on
level-j errors right after the coarse-grid correction of MGM iterations of
the sub-hierarchy that starts at level j, on L_j e = 0.

Bordered Poisson system (Sec. 4.4; our reading): the Richardson steps hold
the multiplier fixed, like the Gauss-Seidel smoother, so a step is
e <- e + omega_q D^-1 (r - L e - b lam); the snapshots come from the
homogeneous bordered iteration (see `snapshots`) and the loss and its
gradient are unchanged.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .colouring import splitmix64

HIDDEN = 64


def counter_uniform(keys: np.ndarray) -> np.ndarray:
    """u(k) = (splitmix64(k) >> 11) * 2^-53 in [0, 1), exactly representable."""
    return (splitmix64(keys.astype(np.uint64)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def power_estimate(L: sp.csr_matrix, steps: int = 20) -> float:
    """lam = |D^-1 L v_k| / |v_k| after `steps` normalised power steps, v_0(i) = u(i) - 1/2."""
    dinv = 1.0 / L.diagonal()
    v = counter_uniform(np.arange(L.shape[0], dtype=np.uint64)) - 0.5
    lam = 0.0
    for _ in range(steps):
        v = v / np.linalg.norm(v)
        w = dinv * (L @ v)
        lam = float(np.linalg.norm(w))
        v = w
    return lam


def cheb_omegas(lam: float, s: int) -> np.ndarray:
    a, b = lam / 4.0, 1.1 * lam
    q = np.arange(1, s + 1)
    theta = (b + a) / 2.0 + (b - a) / 2.0 * np.cos((2 * q - 1) * math.pi / (2 * s))
    return 1.0 / theta


def features(xh: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Per-node features (N x 3n): scaled tangent coordinates and normalised weights."""
    rho = np.sqrt((xh ** 2).sum(axis=2)).max(axis=1)
    xs = xh / rho[:, None, None]
    cw = weights / np.abs(weights[:, :1])
    return np.concatenate([xs.reshape(len(xh), -1), cw], axis=1)


def init_params(n_in: int, s: int, seed: int):
    """Glorot-uniform hidden layers from the counter generator, zero last layer.

    Entry idx (row-major) of the weight of layer l uses key
    seed * 2^32 + l * 2^24 + idx.
    """
    params = []
    dims = [(n_in, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, s)]
    for l, (fi, fo) in enumerate(dims):
        if l < 2:
            keys = np.uint64(seed) * np.uint64(1 << 32) + np.uint64(l << 24) + np.arange(fi * fo, dtype=np.uint64)
            lim = math.sqrt(6.0 / (fi + fo))
            W = ((counter_uniform(keys) * 2.0 - 1.0) * lim).reshape(fi, fo)
        else:
            W = np.zeros((fi, fo))
        params += [W, np.zeros(fo)]
    return params


def mlp_forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    o = h2 @ W3 + b3
    return o, (X, z1, h1, z2, h2)


def mlp_backward(params, cache, do):
    W1, b1, W2, b2, W3, b3 = params
    X, z1, h1, z2, h2 = cache
    dW3 = h2.T @ do
    db3 = do.sum(axis=0)
    dh2 = (do @ W3.T) * (z2 > 0)
    dW2 = h1.T @ dh2
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (z1 > 0)
    dW1 = X.T @ dh1
    db1 = dh1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


def omegas_from_output(o: np.ndarray, wcheb: np.ndarray) -> np.ndarray:
    return wcheb[None, :] * (1.0 + 0.5 * np.tanh(o))


def smooth(L: sp.csr_matrix, omega: np.ndarray, e: np.ndarray, r: np.ndarray | None = None) -> np.ndarray:
    """s Richardson steps e <- e + omega_q D^-1 (r - L e) (r = 0 when None)."""
    dinv = 1.0 / L.diagonal()
    for q in range(omega.shape[1]):
        res = -(L @ e) if r is None else r - L @ e
        e = e + omega[:, q] * dinv * res
    return e


def loss_and_grad_omega(L: sp.csr_matrix, omega: np.ndarray, snaps: np.ndarray):
    """Loss mean_t |L S e_t|^2/|L e_t|^2 and its gradient w.r.t. omega (N x s)."""
    dinv = 1.0 / L.diagonal()
    LT = L.T.tocsr()
    s = omega.shape[1]
    T = snaps.shape[0]
    loss = 0.0
    grad = np.zeros_like(omega)
    for t in range(T):
        e = snaps[t]
        c = float(np.linalg.norm(L @ e) ** 2)
        zs = []
        for q in range(s):
            z = dinv * (L @ e)
            zs.append(z)
            e = e - omega[:, q] * z
        y = L @ e
        loss += float(y @ y) / c / T
        g = 2.0 * (LT @ y) / c / T
        for q in range(s - 1, -1, -1):
            grad[:, q] += -g * zs[q]
            g = g - LT @ (dinv * (omega[:, q] * g))
    return loss, grad


def total_loss_and_grads(params, X, L, snaps, wcheb):
    o, cache = mlp_forward(params, X)
    omega = omegas_from_output(o, wcheb)
    loss, gw = loss_and_grad_omega(L, omega, snaps)
    do = gw * wcheb[None, :] * 0.5 * (1.0 - np.tanh(o) ** 2)
    return loss, mlp_backward(params, cache, do)


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            out.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
        return out


def train(params, X, L, snaps, wcheb, steps, lr=1e-3):
    opt = Adam(params, lr)
    hist = []
    for _ in range(steps):
        loss, grads = total_loss_and_grads(params, X, L, snaps, wcheb)
        hist.append(loss)
        params = opt.step(params, grads)
    return params, hist


def snapshots(H, starts: np.ndarray, iters: int, level: int = 0) -> np.ndarray:
    """Error snapshots of level `level` for training (homogeneous L_j e = 0).

    From each start e (rows of `starts`, level-j vectors), `iters` MGM
    iterations e <- e + M_j(-L_j e) with the Gauss-Seidel cycle of the
    sub-hierarchy from level j; each iteration contributes e + (level-j vector
    right after the coarse correction).

    Bordered Poisson system (Sec. 4.4; our reading): the iteration runs on the
    homogeneous bordered system of level j, [L_j b_j; b_j^T 0] (e, mu) = 0,
    from (start, 0): (e, mu) <- (e, mu) + M_j(-(L_j e + b_j mu), -b_j . e).
    The snapshots are the e parts; the smoother holds mu fixed, so the loss
    is the same function of L_j as for the screened problem."""
    from .vcycle import Fp64Ops, vcycle
    ops = Fp64Ops(H)
    L = H.levels[level].L
    b = H.levels[level].b if H.problem == "poisson" else None
    out = []
    for e0 in starts:
        e = np.array(e0, dtype=np.float64)
        mu = 0.0
        for _ in range(iters):
            cap = []
            if b is None:
                z = vcycle(ops, -(L @ e), None, capture=cap, level=level)
            else:
                z, dmu = vcycle(ops, -(L @ e + b * mu), -float(b @ e), capture=cap, level=level)
                mu += dmu
            out.append(e + cap[0])
            e = e + z
    return np.array(out)


def level_fine_index(H, j: int) -> np.ndarray:
    """Fine-level index of every level-j point (the coarse sets are nested)."""
    idx = np.arange(H.levels[0].N)
    for k in range(j):
        idx = idx[H.levels[k].coarse_idx]
    return idx


def level_features(H, j: int) -> np.ndarray:
    """Features of level j (j = 0: `stencil_features`)."""
    if j == 0:
        return stencil_features(H)
    from .discretize import project_stencils
    from .knn import stencils
    lv = H.levels[j]
    n = min(H.stencils.shape[1], lv.N)
    sten = stencils(lv.xyz, n)
    nrm = H.normals[level_fine_index(H, j)]
    xh = project_stencils(lv.xyz, nrm, sten)
    vals = np.asarray(lv.L[np.repeat(np.arange(lv.N), n), sten.ravel()]).reshape(lv.N, n)
    return features(xh, vals)


def stencil_features(H) -> np.ndarray:
    """Features of the fine level from the hierarchy's stencils and weights."""
    from .discretize import project_stencils
    lv = H.levels[0]
    xh = project_stencils(lv.xyz, H.normals, H.stencils) if hasattr(H, "normals") else None
    return features(xh, H.weights)
