// Learned per-node Chebyshev smoother, one per smoothed level: features,
// spectral estimate, training snapshots, training (MLP forward/backward,
// adjoint of the smoother, Adam) and activation with Gauss-Seidel as the
// fallback.
//
// The smoother (an extension; the paper smooths with Gauss-Seidel, Sec. 4.3):
// s Richardson steps e <- e + omega_{q,i} D^-1 (f - L e) with
// omega_{q,i} = omega_q (1 + 0.5 tanh(o_{q,i})), omega_q = 1/theta_q the
// reciprocal Chebyshev roots on [lam/4, 1.1 lam], lam a 20-step power
// estimate of rho(D^-1 L), and o = MLP(features_i). Features of node i over
// its stencil in distance order: tangent-plane coordinates (Sec. 2.1) divided
// by the stencil radius, and the LBO weights (Sec. 2.2-2.3) divided by
// |c_ii|. Training snapshots: fine-level errors right after the coarse-grid
// correction of MGM iterations on L e = 0 from caller-supplied random starts;
// loss mean_t |L S e_t|^2 / |L e_t|^2.
// A coarse level j has its own smoother of the same form: features from the
// level's own n nearest points (the coarse points are fine points and keep
// their normals) and the entries of the Galerkin operator L_j at those points
// over |L_j(i,i)| (0 off its pattern); snapshots from the cycle of the
// sub-hierarchy that starts at level j, on L_j e = 0.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "ctx.h"
#include "kernels_learned.h"

namespace mgm {

namespace {

constexpr int kPowerSteps = 20;

void ensure_learned_buffers(mgm_ctx* c, int j, int s, int T) {
  DevLevel& d = c->lv[j];
  LearnedLevel& L = c->ls[j];
  const int n = d.n;
  const int nin = L.nin;
  const int np = mlp_param_count(nin, s);
  if (!L.params || L.s != s) {
    L.params = track(c, dalloc<float>(np));
    L.m = track(c, dalloc<float>(np));
    L.v = track(c, dalloc<float>(np));
    L.grad = track(c, dalloc<float>(np));
    L.om64 = track(c, dalloc<double>(size_t(s) * n));
    L.om32 = track(c, dalloc<float>(size_t(s) * n));
    L.O = track(c, dalloc<float>(size_t(n) * s));
    L.dO = track(c, dalloc<float>(size_t(n) * s));
    L.domega = track(c, dalloc<float>(size_t(n) * s));
    L.omt = track(c, dalloc<float>(size_t(n) * s));
    L.wcheb_d = track(c, dalloc<double>(s));
    L.s = s;
  }
  if (!L.H1) {
    L.H1 = track(c, dalloc<float>(size_t(n) * (kHid + 1)));
    L.H2 = track(c, dalloc<float>(size_t(n) * (kHid + 1)));
    L.dH1 = track(c, dalloc<float>(size_t(n) * kHid));
    L.dH2 = track(c, dalloc<float>(size_t(n) * kHid));
    L.e = track(c, dalloc<float>(size_t(2) * n));
    L.y = track(c, dalloc<float>(n));
    L.g = track(c, dalloc<float>(size_t(2) * n));
    L.t = track(c, dalloc<float>(n));
    L.scal = track(c, dalloc<double>(16));
    const int nb = (n + kAtbChunk - 1) / kAtbChunk;
    // partials of the widest product: the first layer's (nin + 1) x 64 or the
    // second's 65 x 64 (the last layer's 65 x s is smaller)
    L.atb = track(c, dalloc<float>(size_t(nb) * std::max(nin + 1, kHid + 1) * kHid));
    L.atb2 = track(c, dalloc<double>(size_t((nb + kColGroup - 1) / kColGroup) * std::max(nin + 1, kHid + 1) * kHid));
  }
  if (!c->e_tmp64) {  // shared by all levels: sized for the fine level
    c->e_tmp64 = track(c, dalloc<double>(c->lv[0].n + 1));
    c->e_tmp32 = track(c, dalloc<float>(c->lv[0].n + 1));
  }
  // snapshots this call makes (T) or keeps from an earlier call (L.T), and the
  // adjoint's step inputs z for each of them and each of the s steps (s may
  // differ from the call that made the snapshots)
  const int tn = std::max(T, L.T);
  if (tn > L.snap_cap) {
    L.snap = track(c, dalloc<float>(size_t(tn) * n));
    L.c = track(c, dalloc<double>(tn));
    L.snap_cap = tn;
  }
  if (size_t(tn) * s * n > L.z_cap) {
    L.z = track(c, dalloc<float>(size_t(tn) * s * n));
    L.z_cap = size_t(tn) * s * n;
  }
}

// features (permuted rows, FP32, with a trailing 1 for the bias)
void build_features(mgm_ctx* c, int j, const std::vector<int32_t>& perm) {
  const HostHierarchy& H = c->H;
  const HostLevel& lv = H.lv[j];
  const int n = lv.n;
  const int ns = std::min(H.ns, n);
  const int nin = 3 * ns;
  std::vector<float> X(size_t(n) * (nin + 1));
  std::vector<int32_t> iperm(n);
  for (int t = 0; t < n; ++t) iperm[perm[t]] = t;
  // stencils, normals and normalised operator entries of level j
  const int32_t* sten = H.stencils.data();
  std::vector<int32_t> csten;
  std::vector<double> cnrm, cval;
  const double* nrm = H.normals.data();
  if (j > 0) {
    std::vector<double> d2;
    knn_search(lv.xyz.data(), n, lv.xyz.data(), n, ns, csten, d2);
    std::vector<int64_t> fidx(H.lv[0].n);  // fine index of each level-k point, k = 0..j
    std::iota(fidx.begin(), fidx.end(), 0);
    for (int k = 0; k < j; ++k) {
      const std::vector<int32_t>& ci = H.lv[k].coarse_idx;
      std::vector<int64_t> nx(ci.size());
      for (size_t t = 0; t < ci.size(); ++t) nx[t] = fidx[ci[t]];
      fidx.swap(nx);
    }
    cnrm.resize(size_t(n) * 3);
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) cnrm[size_t(i) * 3 + a] = H.normals[size_t(fidx[i]) * 3 + a];
    cval.assign(size_t(n) * ns, 0.0);
    parallel_for(n, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e; ++i) {
        const int32_t* cb = lv.L.col.data() + lv.L.ptr[i];
        const int32_t* ce = lv.L.col.data() + lv.L.ptr[i + 1];
        for (int k = 0; k < ns; ++k) {
          const int32_t* it = std::lower_bound(cb, ce, csten[size_t(i) * ns + k]);
          if (it != ce && *it == csten[size_t(i) * ns + k]) cval[size_t(i) * ns + k] = lv.L.val[lv.L.ptr[i] + (it - cb)];
        }
      }
    });
    sten = csten.data();
    nrm = cnrm.data();
  }
  const double* wts = j == 0 ? H.weights.data() : cval.data();
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<double> xh(2 * ns);
    for (int64_t i = b; i < e; ++i) {
      project_stencil(lv.xyz.data(), nrm, i, &sten[size_t(i) * ns], ns, xh.data());
      double rho = 0.0;
      for (int k = 0; k < ns; ++k) rho = std::max(rho, std::sqrt(xh[2 * k] * xh[2 * k] + xh[2 * k + 1] * xh[2 * k + 1]));
      float* row = &X[size_t(iperm[i]) * (nin + 1)];
      for (int k = 0; k < 2 * ns; ++k) row[k] = float(xh[k] / rho);
      const double c0 = std::fabs(wts[size_t(i) * ns]);
      for (int k = 0; k < ns; ++k) row[2 * ns + k] = float(wts[size_t(i) * ns + k] / c0);
      row[nin] = 1.0f;
    }
  });
  c->ls[j].nin = nin;
  c->ls[j].X = track(c, dupload(X));
}

// transposed fine operator (permuted numbering), FP32 values
void build_transpose(mgm_ctx* c, int j) {
  DevLevel& d = c->lv[j];
  LearnedLevel& L = c->ls[j];
  const int n = d.n;
  std::vector<int32_t> col(d.nnz);
  HIPCHECK(hipMemcpy(col.data(), d.col, sizeof(int32_t) * d.nnz, hipMemcpyDeviceToHost));
  Csr A;
  A.nrows = A.ncols = n;
  A.ptr.assign(d.rowlen_prefix.begin(), d.rowlen_prefix.end());
  A.col = col;
  A.val = d.hv;
  Csr T = transpose(A);
  std::vector<float> tv(T.val.begin(), T.val.end());
  L.tptr = track(c, dupload(T.ptr));
  L.tcol = track(c, dupload(T.col));
  L.tval = track(c, dupload(tv));
}

double power_estimate(mgm_ctx* c, int j, hipStream_t st) {
  DevLevel& d = c->lv[j];
  const int n = d.n;
  double* v = c->vecs + 2 * c->ld;
  double* w = c->vecs + 3 * c->ld;
  hipLaunchKernelGGL(k_counter_start, dim3(nblk(n)), dim3(kBlock), 0, st, n, d.perm, v);
  const unsigned g = nblk(int64_t(n) * d.G);
  for (int it = 0; it < kPowerSteps; ++it) {
    mdot(c, n, v, c->ld, 1, v, c->dh, st);
    switch (d.G) {
      case 2: hipLaunchKernelGGL((k_power_step<2>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v64, d.dinv64, c->dh, v, w); break;
      case 4: hipLaunchKernelGGL((k_power_step<4>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v64, d.dinv64, c->dh, v, w); break;
      case 8: hipLaunchKernelGGL((k_power_step<8>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v64, d.dinv64, c->dh, v, w); break;
      default: hipLaunchKernelGGL((k_power_step<16>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v64, d.dinv64, c->dh, v, w); break;
    }
    std::swap(v, w);
  }
  mdot(c, n, v, c->ld, 1, v, c->dh, st);
  to_host(c, c->dh, 1, st);
  return std::sqrt(c->hpin[0]);
}

#define SPMV_F32(G_, n_, W_, ptr_, col_, val_, x_, y_)                                                          \
  switch (G_) {                                                                                                \
    case 2: hipLaunchKernelGGL((k_spmv<float, float, 2, false, false>), dim3(nblk(int64_t(n_) * 2)), dim3(kBlock), 0, st, n_, W_, ptr_, col_, val_, nullptr, x_, y_, nullptr, nullptr); break;   \
    case 4: hipLaunchKernelGGL((k_spmv<float, float, 4, false, false>), dim3(nblk(int64_t(n_) * 4)), dim3(kBlock), 0, st, n_, W_, ptr_, col_, val_, nullptr, x_, y_, nullptr, nullptr); break;   \
    case 8: hipLaunchKernelGGL((k_spmv<float, float, 8, false, false>), dim3(nblk(int64_t(n_) * 8)), dim3(kBlock), 0, st, n_, W_, ptr_, col_, val_, nullptr, x_, y_, nullptr, nullptr); break;   \
    default: hipLaunchKernelGGL((k_spmv<float, float, 16, false, false>), dim3(nblk(int64_t(n_) * 16)), dim3(kBlock), 0, st, n_, W_, ptr_, col_, val_, nullptr, x_, y_, nullptr, nullptr); break; \
  }

void fdot(mgm_ctx* c, int n, const float* x, const float* y, double* out, hipStream_t st) {
  const int nb = std::min(kRedBlocks, std::max(1, (n + 2047) / 2048));
  hipLaunchKernelGGL(k_fdot_partial, dim3(nb), dim3(kBlock), 0, st, n, x, y, c->kpart);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, 1, nb, c->kpart, out);
}

void atb(mgm_ctx* c, LearnedLevel& L, int n, int ka, int kb, const float* A, const float* B, float* out, hipStream_t st) {
  if (ka > kAtbMaxK || kb > 64) throw Error(MGM_E_ARG, "learned smoother: layer too wide");
  const int nb = (n + kAtbChunk - 1) / kAtbChunk;
  if (kb <= 16) hipLaunchKernelGGL((k_atb_partial<1>), dim3(nb), dim3(64 * kAtbWaves), 0, st, n, ka, kb, A, B, L.atb);
  else hipLaunchKernelGGL((k_atb_partial<4>), dim3(nb), dim3(64 * kAtbWaves), 0, st, n, ka, kb, A, B, L.atb);
  const int ng = (nb + kColGroup - 1) / kColGroup;
  hipLaunchKernelGGL(k_reduce_cols_group, dim3(nblk(ka * kb), ng), dim3(kBlock), 0, st, nb, ka * kb, L.atb, L.atb2);
  hipLaunchKernelGGL(k_reduce_cols, dim3(nblk(ka * kb)), dim3(kBlock), 0, st, ng, ka * kb, L.atb2, out);
}

// one loss/gradient evaluation (and an Adam step when `update`); the loss of
// this evaluation is accumulated into loss_slot (device)
void train_step(mgm_ctx* c, int j, bool update, double* loss_slot, float lr, hipStream_t st) {
  DevLevel& d = c->lv[j];
  LearnedLevel& L = c->ls[j];
  const int n = d.n, s = L.s, nin = L.nin, T = L.T;
  if (T > L.snap_cap || size_t(T) * s * n > L.z_cap) throw Error(MGM_E_ARG, "learned smoother: training buffers too small");
  const int np = mlp_param_count(nin, s);
  const unsigned mlp_blocks = unsigned((n + kMlpNodes - 1) / kMlpNodes);
  hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_blocks), dim3(64 * kMlpWaves), 0, st, n, nin, s, L.X, L.params, L.O,
                     L.H1, L.H2);
  hipLaunchKernelGGL((k_omega<float>), dim3(nblk(n)), dim3(kBlock), 0, st, n, s, L.O, L.wcheb_d, L.omt);
  hipLaunchKernelGGL((k_fill<float>), dim3(nblk(int64_t(n) * s)), dim3(kBlock), 0, st, n * s, L.domega, 0.0f);
  hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(kBlock), 0, st, 1, loss_slot, 0.0);
  const unsigned g = nblk(int64_t(n) * d.G);
  for (int t = 0; t < T; ++t) {
    const float* ein = L.snap + size_t(t) * n;
    float* bufs[2] = {L.e, L.e + n};
    for (int q = 0; q < s; ++q) {
      float* eout = bufs[q & 1];
      float* z = L.z + (size_t(t) * s + q) * n;
      const float* om = L.omt + size_t(q) * n;
      switch (d.G) {
        case 2: hipLaunchKernelGGL((k_train_step<2>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v32, d.dinv32, om, ein, eout, z); break;
        case 4: hipLaunchKernelGGL((k_train_step<4>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v32, d.dinv32, om, ein, eout, z); break;
        case 8: hipLaunchKernelGGL((k_train_step<8>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v32, d.dinv32, om, ein, eout, z); break;
        default: hipLaunchKernelGGL((k_train_step<16>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v32, d.dinv32, om, ein, eout, z); break;
      }
      ein = eout;
    }
    SPMV_F32(d.G, n, d.W, d.rowptr, d.col, d.v32, ein, L.y);
    fdot(c, n, L.y, L.y, L.scal, st);
    hipLaunchKernelGGL(k_loss_acc, dim3(1), dim3(64), 0, st, L.scal, L.c + t, 1.0 / T, loss_slot);
    // g = 2 L^T y / (c_t T)
    float* gb[2] = {L.g, L.g + n};
    SPMV_F32(d.G, n, 0, L.tptr, L.tcol, L.tval, L.y, gb[0]);
    hipLaunchKernelGGL(k_scale_ct, dim3(nblk(n)), dim3(kBlock), 0, st, n, L.c + t, 2.0 / T, gb[0]);
    int cur = 0;
    for (int q = s - 1; q >= 0; --q) {
      const float* z = L.z + (size_t(t) * s + q) * n;
      hipLaunchKernelGGL(k_adj_accum, dim3(nblk(n)), dim3(kBlock), 0, st, n, gb[cur], z, d.dinv32, L.omt + size_t(q) * n,
                         L.domega + size_t(q) * n, L.t);
      if (q > 0) {
        switch (d.G) {
          case 2: hipLaunchKernelGGL((k_xmAt<2>), dim3(g), dim3(kBlock), 0, st, n, 0, L.tptr, L.tcol, L.tval, gb[cur], L.t, gb[1 - cur]); break;
          case 4: hipLaunchKernelGGL((k_xmAt<4>), dim3(g), dim3(kBlock), 0, st, n, 0, L.tptr, L.tcol, L.tval, gb[cur], L.t, gb[1 - cur]); break;
          case 8: hipLaunchKernelGGL((k_xmAt<8>), dim3(g), dim3(kBlock), 0, st, n, 0, L.tptr, L.tcol, L.tval, gb[cur], L.t, gb[1 - cur]); break;
          default: hipLaunchKernelGGL((k_xmAt<16>), dim3(g), dim3(kBlock), 0, st, n, 0, L.tptr, L.tcol, L.tval, gb[cur], L.t, gb[1 - cur]); break;
        }
        cur = 1 - cur;
      }
    }
  }
  hipLaunchKernelGGL(k_mlp_backward, dim3(mlp_blocks), dim3(64 * kMlpWaves), 0, st, n, nin, s, L.params, L.O,
                     L.domega, L.wcheb_d, L.H1, L.H2, L.dO, L.dH1, L.dH2);
  atb(c, L, n, nin + 1, kHid, L.X, L.dH1, L.grad, st);
  atb(c, L, n, kHid + 1, kHid, L.H1, L.dH2, L.grad + (nin + 1) * kHid, st);
  atb(c, L, n, kHid + 1, s, L.H2, L.dO, L.grad + (nin + 1) * kHid + (kHid + 1) * kHid, st);
  if (update) {
    L.adam_t++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, float(L.adam_t)), c2 = 1.0f - std::pow(b2, float(L.adam_t));
    hipLaunchKernelGGL(k_adam, dim3(nblk(np)), dim3(kBlock), 0, st, np, L.params, L.grad, L.m, L.v, lr, b1,
                       b2, 1e-8f, c1, c2);
  }
}

// inference step weights from the current parameters
void compute_omega(mgm_ctx* c, int j, hipStream_t st) {
  DevLevel& d = c->lv[j];
  LearnedLevel& L = c->ls[j];
  const int n = d.n, s = L.s, nin = L.nin;
  hipLaunchKernelGGL(k_mlp_forward, dim3(unsigned((n + kMlpNodes - 1) / kMlpNodes)), dim3(64 * kMlpWaves), 0, st, n,
                     nin, s, L.X, L.params, L.O, (float*)nullptr, (float*)nullptr);
  hipLaunchKernelGGL((k_omega<double>), dim3(nblk(n)), dim3(kBlock), 0, st, n, s, L.O, L.wcheb_d, L.om64);
  hipLaunchKernelGGL((k_omega<float>), dim3(nblk(n)), dim3(kBlock), 0, st, n, s, L.O, L.wcheb_d, L.om32);
}

// y = A_j x (FP64, permuted order; the fine level through the outer operator;
// bordered: n_j + 1 entries, the multiplier at index n_j)
void apply_level(mgm_ctx* c, int j, const double* x, double* y, hipStream_t st) {
  if (j == 0) apply_A(c, x, y, st);
  else spmv_level64(c, j, x, y, st);
}

// z = M_j v (FP64, permuted order): the full cycle on the fine level, the
// sub-hierarchy's cycle on a coarse level
void precond_at(mgm_ctx* c, int j, const double* v, double* z, hipStream_t st) {
  if (j == 0) precond(c, v, z, nullptr, st);
  else precond_level(c, j, v, z, st);
}

// convergence factor of the stationary MGM iteration on A_j e = 0 from `e0`
// (permuted FP64; bordered: n_j + 1 entries, the multiplier last):
// (|A_j e_k| / |A_j e_0|)^(1/k)
double stationary_rate(mgm_ctx* c, int j, const double* e0, int k, hipStream_t st) {
  DevLevel& d = c->lv[j];
  const int n = d.n + (c->p.problem == MGM_POISSON ? 1 : 0);
  double* e = c->vecs + 4 * c->ld;
  double* r = c->vecs + 5 * c->ld;
  double* z = c->vecs + 6 * c->ld;
  HIPCHECK(hipMemcpyAsync(e, e0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  double n0 = 0.0, nk = 0.0;
  for (int it = 0; it <= k; ++it) {
    apply_level(c, j, e, r, st);
    mdot(c, n, r, c->ld, 1, r, c->dh, st);
    to_host(c, c->dh, 1, st);
    if (it == 0) n0 = std::sqrt(c->hpin[0]);
    if (it == k) {
      nk = std::sqrt(c->hpin[0]);
      break;
    }
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(kBlock), 0, st, n, -1.0, r, 0.0, r, r);
    precond_at(c, j, r, z, st);
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(kBlock), 0, st, n, 1.0, e, 1.0, z, e);
  }
  return n0 > 0.0 ? std::pow(nk / n0, 1.0 / k) : 0.0;
}

void init_params_counter(mgm_ctx* c, int j, uint64_t seed, hipStream_t st) {
  LearnedLevel& L = c->ls[j];
  const int nin = L.nin, s = L.s;
  std::vector<float> p(mlp_param_count(nin, s), 0.0f);
  auto u = [](uint64_t k) {
    uint64_t z = k + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return double(z >> 11) * 0x1.0p-53;
  };
  // layer l (0, 1) weight entry idx (row-major, fan_in x 64) uses key seed*2^32 + l*2^24 + idx;
  // biases and the last layer start at zero
  const int fin[2] = {nin, kHid};
  size_t off = 0;
  for (int l = 0; l < 2; ++l) {
    const double lim = std::sqrt(6.0 / (fin[l] + kHid));
    for (int idx = 0; idx < fin[l] * kHid; ++idx)
      p[off + idx] = float((u(seed * (uint64_t(1) << 32) + (uint64_t(l) << 24) + uint64_t(idx)) * 2.0 - 1.0) * lim);
    off += size_t(fin[l] + 1) * kHid;
  }
  HIPCHECK(hipMemcpyAsync(L.params, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemsetAsync(L.m, 0, p.size() * sizeof(float), st));
  HIPCHECK(hipMemsetAsync(L.v, 0, p.size() * sizeof(float), st));
  L.adam_t = 0;
}

void set_active(mgm_ctx* c, int j, bool on) {
  LearnedLevel& L = c->ls[j];
  if (L.active != on) {
    L.active = on;
    invalidate_graphs(c);
  }
}

void ensure_levels(mgm_ctx* c) {
  const size_t nl = c->lv.size() - 1;  // smoothed levels
  if (c->ls.size() < nl) c->ls.resize(nl);
}

}  // namespace

}  // namespace mgm

using namespace mgm;

extern "C" {

mgm_status mgm_train_smoother(mgm_handle h, const mgm_train_opts* o, const double* d_starts, mgm_train_info* info,
                              double* h_loss_hist, void* stream) {
  if (!h || !o || !info || o->s < 1 || o->s > 8 || o->steps < 0 || o->n_starts < 0 || o->iters_per_start < 0 ||
      o->activate < 0 || o->activate > 2 || (o->n_starts > 0 && !d_starts)) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int j = o->level;
    if (j < 0 || j + 1 >= int(h->lv.size())) throw Error(MGM_E_ARG, "learned smoother: level out of range");
    ensure_levels(h);
    LearnedLevel& L = h->ls[j];
    DevLevel& d = h->lv[j];
    const int n = d.n;
    // bordered problems iterate on the level's bordered system: the
    // multiplier rides at index n (zero in every start)
    const bool bord = h->p.problem == MGM_POISSON;
    const int nv = n + (bord ? 1 : 0);
    ensure_ws(h, 1);
    build_precision(h, MGM_FP32);
    build_precision(h, MGM_FP64);
    std::vector<int32_t> perm(n);
    if (d.perm) HIPCHECK(hipMemcpy(perm.data(), d.perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    else std::iota(perm.begin(), perm.end(), 0);
    if (!L.X) {
      build_features(h, j, perm);
      build_transpose(h, j);
    }
    // the gradient products take at most kAtbMaxK rows of the first layer
    if (L.nin + 1 > kAtbMaxK) throw Error(MGM_E_ARG, "learned smoother: layer too wide (stencils above 66 points)");
    const bool was_active = L.active;
    const bool fresh = !L.params || L.s != o->s;
    const int T = o->n_starts * o->iters_per_start;
    ensure_learned_buffers(h, j, o->s, std::max(T, 1));
    *info = mgm_train_info{};
    // spectral estimate and Chebyshev step weights
    L.lam = power_estimate(h, j, st);
    const double a = L.lam / 4.0, b = 1.1 * L.lam;
    L.wcheb.resize(o->s);
    for (int q = 1; q <= o->s; ++q)
      L.wcheb[q - 1] = 1.0 / ((b + a) / 2.0 + (b - a) / 2.0 * std::cos((2.0 * q - 1.0) * M_PI / (2.0 * o->s)));
    HIPCHECK(hipMemcpyAsync(L.wcheb_d, L.wcheb.data(), sizeof(double) * o->s, hipMemcpyHostToDevice, st));
    info->lam = L.lam;
    if (o->init || fresh) init_params_counter(h, j, o->seed, st);
    // snapshots with the Gauss-Seidel cycle (every level) in FP64
    std::vector<char> mask(h->ls.size());
    for (size_t k = 0; k < h->ls.size(); ++k) mask[k] = h->ls[k].active;
    if (T > 0) {
      for (size_t k = 0; k < h->ls.size(); ++k) set_active(h, int(k), false);
      const int prec = h->p.precision;
      h->p.precision = MGM_FP64;
      double* e = h->vecs + 4 * h->ld;
      double* r = h->vecs + 5 * h->ld;
      double* z = h->vecs + 6 * h->ld;
      double* cap = h->vecs + 7 * h->ld;
      int t = 0;
      for (int s0 = 0; s0 < o->n_starts; ++s0) {
        hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(n)), dim3(kBlock), 0, st, n, d.perm, d_starts + size_t(s0) * n,
                           e, (double*)nullptr);
        if (bord) hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(kBlock), 0, st, 1, e + n, 0.0);
        for (int it = 0; it < o->iters_per_start; ++it, ++t) {
          apply_level(h, j, e, r, st);
          hipLaunchKernelGGL(k_axpby, dim3(nblk(nv)), dim3(kBlock), 0, st, nv, -1.0, r, 0.0, r, r);
          h->capture = cap;
          h->capture_level = j;
          precond_at(h, j, r, z, st);
          h->capture = nullptr;
          h->capture_level = 0;
          hipLaunchKernelGGL(k_add_cast, dim3(nblk(n)), dim3(kBlock), 0, st, n, e, cap, L.snap + size_t(t) * n);
          hipLaunchKernelGGL(k_axpby, dim3(nblk(nv)), dim3(kBlock), 0, st, nv, 1.0, e, 1.0, z, e);
          // c_t = |L e_t|^2 in the training precision
          SPMV_F32(d.G, n, d.W, d.rowptr, d.col, d.v32, L.snap + size_t(t) * n, L.y);
          fdot(h, n, L.y, L.y, L.c + t, st);
        }
      }
      h->p.precision = prec;
      L.T = T;
      for (size_t k = 0; k < h->ls.size(); ++k) set_active(h, int(k), mask[k] != 0);
    }
    if (L.T < 1 && o->steps > 0) throw Error(MGM_E_ARG, "learned smoother: no snapshots");
    // training
    if (o->steps > 0) {
      if (!L.loss || o->steps + 1 > L.steps_cap) {
        L.loss = track(h, dalloc<double>(o->steps + 1));
        L.steps_cap = o->steps + 1;
      }
      for (int it = 0; it < o->steps; ++it) train_step(h, j, true, L.loss + it, float(o->lr), st);
      train_step(h, j, false, L.loss + o->steps, float(o->lr), st);
      std::vector<double> hist(o->steps + 1);
      HIPCHECK(hipMemcpyAsync(hist.data(), L.loss, sizeof(double) * hist.size(), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      info->loss_first = hist.front();
      info->loss_last = hist.back();
      if (h_loss_hist) std::copy(hist.begin(), hist.end(), h_loss_hist);
    }
    compute_omega(h, j, st);
    // activation: compare stationary convergence factors from the first start
    // (the other levels keep their smoothers)
    if (o->activate == 2) {
      set_active(h, j, true);
    } else if (o->activate == 1 && o->n_starts > 0) {
      double* e0 = h->vecs + 8 * h->ld;
      hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(n)), dim3(kBlock), 0, st, n, d.perm, d_starts, e0,
                         (double*)nullptr);
      if (bord) hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(kBlock), 0, st, 1, e0 + n, 0.0);
      set_active(h, j, false);
      info->rate_gs = stationary_rate(h, j, e0, 6, st);
      set_active(h, j, true);
      info->rate_learned = stationary_rate(h, j, e0, 6, st);
      set_active(h, j, info->rate_learned < info->rate_gs);
    } else {
      set_active(h, j, o->activate == 0 ? false : was_active);
    }
    info->active = L.active ? 1 : 0;
    HIPCHECK(hipStreamSynchronize(st));
  });
}

mgm_status mgm_smoother_params(mgm_handle h, int32_t level, int32_t set, float* h_params, int64_t* len) {
  if (!h || !len) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    if (level < 0 || level >= int(h->ls.size()) || !h->ls[level].params)
      throw Error(MGM_E_ARG, "learned smoother not prepared on this level (call mgm_train_smoother first)");
    LearnedLevel& L = h->ls[level];
    const int64_t np = mlp_param_count(L.nin, L.s);
    if (!h_params) {
      *len = np;
      return;
    }
    if (*len < np) throw Error(MGM_E_ARG, "parameter buffer too small");
    if (set) {
      HIPCHECK(hipMemcpy(L.params, h_params, np * sizeof(float), hipMemcpyHostToDevice));
      HIPCHECK(hipMemset(L.m, 0, np * sizeof(float)));
      HIPCHECK(hipMemset(L.v, 0, np * sizeof(float)));
      L.adam_t = 0;
      compute_omega(h, level, nullptr);
      HIPCHECK(hipDeviceSynchronize());
    } else {
      HIPCHECK(hipMemcpy(h_params, L.params, np * sizeof(float), hipMemcpyDeviceToHost));
    }
    *len = np;
  });
}

mgm_status mgm_smoother_grad(mgm_handle h, int32_t level, float* h_grad, double* loss, void* stream) {
  if (!h || !loss) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (level < 0 || level >= int(h->ls.size()) || !h->ls[level].params || h->ls[level].T < 1)
      throw Error(MGM_E_ARG, "learned smoother has no snapshots on this level");
    LearnedLevel& L = h->ls[level];
    ensure_ws(h, 1);
    if (!L.loss) {
      L.loss = track(h, dalloc<double>(2));
      L.steps_cap = 2;
    }
    train_step(h, level, false, L.loss, 0.0f, st);
    const int64_t np = mlp_param_count(L.nin, L.s);
    if (h_grad) HIPCHECK(hipMemcpyAsync(h_grad, L.grad, np * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(loss, L.loss, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
  });
}

mgm_status mgm_set_smoother(mgm_handle h, int32_t level_mask) {
  if (!h) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    const int nl = int(h->lv.size()) - 1;
    if (level_mask < 0 || (nl < 31 && (level_mask >> nl) != 0)) throw Error(MGM_E_ARG, "level mask names a level without a smoother");
    ensure_levels(h);
    for (int j = 0; j < nl; ++j)
      if (((level_mask >> j) & 1) && !h->ls[j].om64) throw Error(MGM_E_ARG, "learned smoother not trained on a level of the mask");
    for (int j = 0; j < nl; ++j) set_active(h, j, ((level_mask >> j) & 1) != 0);
  });
}

}  // extern "C"
