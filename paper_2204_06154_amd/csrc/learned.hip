// Learned per-node Chebyshev smoother on the fine level: features, spectral
// estimate, training snapshots, training (MLP forward/backward, adjoint of the
// smoother, Adam) and activation with Gauss-Seidel as the fallback.
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
#include <algorithm>
#include <cmath>

#include "ctx.h"
#include "kernels_learned.h"

namespace mgm {

namespace {

constexpr int kPowerSteps = 20;

void ensure_learned_buffers(mgm_ctx* c, int s, int T) {
  DevLevel& d = c->lv[0];
  const int n = d.n;
  const int nin = c->ls_nin;
  const int np = mlp_param_count(nin, s);
  if (!c->ls_params || c->ls_s != s) {
    c->ls_params = track(c, dalloc<float>(np));
    c->ls_m = track(c, dalloc<float>(np));
    c->ls_v = track(c, dalloc<float>(np));
    c->ls_grad = track(c, dalloc<float>(np));
    c->ls_om64 = track(c, dalloc<double>(size_t(s) * n));
    c->ls_om32 = track(c, dalloc<float>(size_t(s) * n));
    c->ls_O = track(c, dalloc<float>(size_t(n) * s));
    c->ls_dO = track(c, dalloc<float>(size_t(n) * s));
    c->ls_domega = track(c, dalloc<float>(size_t(n) * s));
    c->ls_omt = track(c, dalloc<float>(size_t(n) * s));
    c->ls_wcheb_d = track(c, dalloc<double>(s));
    c->ls_s = s;
  }
  if (!c->ls_H1) {
    c->ls_H1 = track(c, dalloc<float>(size_t(n) * (kHid + 1)));
    c->ls_H2 = track(c, dalloc<float>(size_t(n) * (kHid + 1)));
    c->ls_dH1 = track(c, dalloc<float>(size_t(n) * kHid));
    c->ls_dH2 = track(c, dalloc<float>(size_t(n) * kHid));
    c->ls_e = track(c, dalloc<float>(size_t(2) * n));
    c->ls_y = track(c, dalloc<float>(n));
    c->ls_g = track(c, dalloc<float>(size_t(2) * n));
    c->ls_t = track(c, dalloc<float>(n));
    c->e_tmp64 = track(c, dalloc<double>(n + 1));
    c->e_tmp32 = track(c, dalloc<float>(n + 1));
    c->ls_scal = track(c, dalloc<double>(16));
    const int nb = (n + kAtbChunk - 1) / kAtbChunk;
    c->ls_atb = track(c, dalloc<float>(size_t(nb) * (nin + 1) * kHid));
  }
  if (T > c->ls_T) {
    c->ls_snap = track(c, dalloc<float>(size_t(T) * n));
    c->ls_z = track(c, dalloc<float>(size_t(T) * s * n));
    c->ls_c = track(c, dalloc<double>(T));
    c->ls_T = T;
  }
}

// features (permuted rows, FP32, with a trailing 1 for the bias)
void build_features(mgm_ctx* c, const std::vector<int32_t>& perm) {
  const HostHierarchy& H = c->H;
  const int n = H.lv[0].n, ns = H.ns;
  const int nin = 3 * ns;
  std::vector<float> X(size_t(n) * (nin + 1));
  std::vector<int32_t> iperm(n);
  for (int t = 0; t < n; ++t) iperm[perm[t]] = t;
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<double> xh(2 * ns);
    for (int64_t i = b; i < e; ++i) {
      project_stencil(H.lv[0].xyz.data(), H.normals.data(), i, &H.stencils[size_t(i) * ns], ns, xh.data());
      double rho = 0.0;
      for (int j = 0; j < ns; ++j) rho = std::max(rho, std::sqrt(xh[2 * j] * xh[2 * j] + xh[2 * j + 1] * xh[2 * j + 1]));
      float* row = &X[size_t(iperm[i]) * (nin + 1)];
      for (int j = 0; j < 2 * ns; ++j) row[j] = float(xh[j] / rho);
      const double c0 = std::fabs(H.weights[size_t(i) * ns]);
      for (int j = 0; j < ns; ++j) row[2 * ns + j] = float(H.weights[size_t(i) * ns + j] / c0);
      row[nin] = 1.0f;
    }
  });
  c->ls_nin = nin;
  c->ls_X = track(c, dupload(X));
}

// transposed fine operator (permuted numbering), FP32 values
void build_transpose(mgm_ctx* c) {
  DevLevel& d = c->lv[0];
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
  c->ls_tptr = track(c, dupload(T.ptr));
  c->ls_tcol = track(c, dupload(T.col));
  c->ls_tval = track(c, dupload(tv));
}

double power_estimate(mgm_ctx* c, hipStream_t st) {
  DevLevel& d = c->lv[0];
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

void atb(mgm_ctx* c, int n, int ka, int kb, const float* A, const float* B, float* out, hipStream_t st) {
  if (ka > kAtbMaxK || kb > kAtbMaxK || ka * kb > 24 * kBlock) throw Error(MGM_E_ARG, "learned smoother: layer too wide");
  const int nb = (n + kAtbChunk - 1) / kAtbChunk;
  hipLaunchKernelGGL(k_atb_partial, dim3(nb), dim3(kBlock), 0, st, n, ka, kb, A, B, c->ls_atb);
  hipLaunchKernelGGL(k_reduce_cols, dim3(nblk(ka * kb)), dim3(kBlock), 0, st, nb, ka * kb, c->ls_atb, out);
}

// one loss/gradient evaluation (and an Adam step when `update`); the loss of
// this evaluation is accumulated into loss_slot (device)
void train_step(mgm_ctx* c, bool update, double* loss_slot, float lr, hipStream_t st) {
  DevLevel& d = c->lv[0];
  const int n = d.n, s = c->ls_s, nin = c->ls_nin, T = c->ls_T;
  const int np = mlp_param_count(nin, s);
  const size_t lds = size_t(np) * sizeof(float);
  hipLaunchKernelGGL(k_mlp_forward, dim3(nblk(n)), dim3(kBlock), lds, st, n, nin, s, c->ls_X, c->ls_params, c->ls_O,
                     c->ls_H1, c->ls_H2);
  hipLaunchKernelGGL((k_omega<float>), dim3(nblk(n)), dim3(kBlock), 0, st, n, s, c->ls_O, c->ls_wcheb_d, c->ls_omt);
  hipLaunchKernelGGL((k_fill<float>), dim3(nblk(int64_t(n) * s)), dim3(kBlock), 0, st, n * s, c->ls_domega, 0.0f);
  hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(kBlock), 0, st, 1, loss_slot, 0.0);
  const unsigned g = nblk(int64_t(n) * d.G);
  for (int t = 0; t < T; ++t) {
    const float* ein = c->ls_snap + size_t(t) * n;
    float* bufs[2] = {c->ls_e, c->ls_e + n};
    for (int q = 0; q < s; ++q) {
      float* eout = bufs[q & 1];
      float* z = c->ls_z + (size_t(t) * s + q) * n;
      const float* om = c->ls_omt + size_t(q) * n;
      switch (d.G) {
        case 2: hipLaunchKernelGGL((k_train_step<2>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v32, d.dinv32, om, ein, eout, z); break;
        case 4: hipLaunchKernelGGL((k_train_step<4>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v32, d.dinv32, om, ein, eout, z); break;
        case 8: hipLaunchKernelGGL((k_train_step<8>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v32, d.dinv32, om, ein, eout, z); break;
        default: hipLaunchKernelGGL((k_train_step<16>), dim3(g), dim3(kBlock), 0, st, n, d.W, d.rowptr, d.col, d.v32, d.dinv32, om, ein, eout, z); break;
      }
      ein = eout;
    }
    SPMV_F32(d.G, n, d.W, d.rowptr, d.col, d.v32, ein, c->ls_y);
    fdot(c, n, c->ls_y, c->ls_y, c->ls_scal, st);
    hipLaunchKernelGGL(k_loss_acc, dim3(1), dim3(64), 0, st, c->ls_scal, c->ls_c + t, 1.0 / T, loss_slot);
    // g = 2 L^T y / (c_t T)
    float* gb[2] = {c->ls_g, c->ls_g + n};
    SPMV_F32(d.G, n, 0, c->ls_tptr, c->ls_tcol, c->ls_tval, c->ls_y, gb[0]);
    hipLaunchKernelGGL(k_scale_ct, dim3(nblk(n)), dim3(kBlock), 0, st, n, c->ls_c + t, 2.0 / T, gb[0]);
    int cur = 0;
    for (int q = s - 1; q >= 0; --q) {
      const float* z = c->ls_z + (size_t(t) * s + q) * n;
      hipLaunchKernelGGL(k_adj_accum, dim3(nblk(n)), dim3(kBlock), 0, st, n, gb[cur], z, d.dinv32, c->ls_omt + size_t(q) * n,
                         c->ls_domega + size_t(q) * n, c->ls_t);
      if (q > 0) {
        switch (d.G) {
          case 2: hipLaunchKernelGGL((k_xmAt<2>), dim3(g), dim3(kBlock), 0, st, n, 0, c->ls_tptr, c->ls_tcol, c->ls_tval, gb[cur], c->ls_t, gb[1 - cur]); break;
          case 4: hipLaunchKernelGGL((k_xmAt<4>), dim3(g), dim3(kBlock), 0, st, n, 0, c->ls_tptr, c->ls_tcol, c->ls_tval, gb[cur], c->ls_t, gb[1 - cur]); break;
          case 8: hipLaunchKernelGGL((k_xmAt<8>), dim3(g), dim3(kBlock), 0, st, n, 0, c->ls_tptr, c->ls_tcol, c->ls_tval, gb[cur], c->ls_t, gb[1 - cur]); break;
          default: hipLaunchKernelGGL((k_xmAt<16>), dim3(g), dim3(kBlock), 0, st, n, 0, c->ls_tptr, c->ls_tcol, c->ls_tval, gb[cur], c->ls_t, gb[1 - cur]); break;
        }
        cur = 1 - cur;
      }
    }
  }
  hipLaunchKernelGGL(k_mlp_backward, dim3(nblk(n)), dim3(kBlock), lds, st, n, nin, s, c->ls_params, c->ls_O, c->ls_domega,
                     c->ls_wcheb_d, c->ls_H1, c->ls_H2, c->ls_dO, c->ls_dH1, c->ls_dH2);
  atb(c, n, nin + 1, kHid, c->ls_X, c->ls_dH1, c->ls_grad, st);
  atb(c, n, kHid + 1, kHid, c->ls_H1, c->ls_dH2, c->ls_grad + (nin + 1) * kHid, st);
  atb(c, n, kHid + 1, s, c->ls_H2, c->ls_dO, c->ls_grad + (nin + 1) * kHid + (kHid + 1) * kHid, st);
  if (update) {
    c->ls_adam_t++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, float(c->ls_adam_t)), c2 = 1.0f - std::pow(b2, float(c->ls_adam_t));
    hipLaunchKernelGGL(k_adam, dim3(nblk(np)), dim3(kBlock), 0, st, np, c->ls_params, c->ls_grad, c->ls_m, c->ls_v, lr, b1,
                       b2, 1e-8f, c1, c2);
  }
}

// inference step weights from the current parameters
void compute_omega(mgm_ctx* c, hipStream_t st) {
  DevLevel& d = c->lv[0];
  const int n = d.n, s = c->ls_s, nin = c->ls_nin;
  const size_t lds = size_t(mlp_param_count(nin, s)) * sizeof(float);
  hipLaunchKernelGGL(k_mlp_forward, dim3(nblk(n)), dim3(kBlock), lds, st, n, nin, s, c->ls_X, c->ls_params, c->ls_O,
                     (float*)nullptr, (float*)nullptr);
  hipLaunchKernelGGL((k_omega<double>), dim3(nblk(n)), dim3(kBlock), 0, st, n, s, c->ls_O, c->ls_wcheb_d, c->ls_om64);
  hipLaunchKernelGGL((k_omega<float>), dim3(nblk(n)), dim3(kBlock), 0, st, n, s, c->ls_O, c->ls_wcheb_d, c->ls_om32);
}

// convergence factor of the stationary MGM iteration on L e = 0 from `e0`
// (permuted FP64): (|L e_k| / |L e_0|)^(1/k)
double stationary_rate(mgm_ctx* c, const double* e0, int k, hipStream_t st) {
  DevLevel& d = c->lv[0];
  const int n = d.n;
  double* e = c->vecs + 4 * c->ld;
  double* r = c->vecs + 5 * c->ld;
  double* z = c->vecs + 6 * c->ld;
  HIPCHECK(hipMemcpyAsync(e, e0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  double n0 = 0.0, nk = 0.0;
  for (int it = 0; it <= k; ++it) {
    apply_A(c, e, r, st);
    mdot(c, n, r, c->ld, 1, r, c->dh, st);
    to_host(c, c->dh, 1, st);
    if (it == 0) n0 = std::sqrt(c->hpin[0]);
    if (it == k) {
      nk = std::sqrt(c->hpin[0]);
      break;
    }
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(kBlock), 0, st, n, -1.0, r, 0.0, r, r);
    precond(c, r, z, nullptr, st);
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(kBlock), 0, st, n, 1.0, e, 1.0, z, e);
  }
  return n0 > 0.0 ? std::pow(nk / n0, 1.0 / k) : 0.0;
}

void init_params_counter(mgm_ctx* c, uint64_t seed, hipStream_t st) {
  const int nin = c->ls_nin, s = c->ls_s;
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
  HIPCHECK(hipMemcpyAsync(c->ls_params, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemsetAsync(c->ls_m, 0, p.size() * sizeof(float), st));
  HIPCHECK(hipMemsetAsync(c->ls_v, 0, p.size() * sizeof(float), st));
  c->ls_adam_t = 0;
}

void set_active(mgm_ctx* c, bool on) {
  if (c->ls_active != on) {
    c->ls_active = on;
    invalidate_graphs(c);
  }
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
    if (h->p.problem != MGM_SCREENED) throw Error(MGM_E_ARG, "learned smoother: screened problems only");
    DevLevel& d = h->lv[0];
    const int n = d.n;
    ensure_ws(h, 1);
    build_precision(h, MGM_FP32);
    std::vector<int32_t> perm(n);
    HIPCHECK(hipMemcpy(perm.data(), d.perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    if (!h->ls_X) {
      build_features(h, perm);
      build_transpose(h);
    }
    const bool was_active = h->ls_active;
    const bool fresh = !h->ls_params || h->ls_s != o->s;
    const int T = o->n_starts * o->iters_per_start;
    ensure_learned_buffers(h, o->s, std::max(T, 1));
    *info = mgm_train_info{};
    // spectral estimate and Chebyshev step weights
    h->ls_lam = power_estimate(h, st);
    const double a = h->ls_lam / 4.0, b = 1.1 * h->ls_lam;
    h->ls_wcheb.resize(o->s);
    for (int q = 1; q <= o->s; ++q)
      h->ls_wcheb[q - 1] = 1.0 / ((b + a) / 2.0 + (b - a) / 2.0 * std::cos((2.0 * q - 1.0) * M_PI / (2.0 * o->s)));
    HIPCHECK(hipMemcpyAsync(h->ls_wcheb_d, h->ls_wcheb.data(), sizeof(double) * o->s, hipMemcpyHostToDevice, st));
    info->lam = h->ls_lam;
    if (o->init || fresh) init_params_counter(h, o->seed, st);
    // snapshots with the Gauss-Seidel V-cycle in FP64
    if (T > 0) {
      set_active(h, false);
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
        for (int it = 0; it < o->iters_per_start; ++it, ++t) {
          apply_A(h, e, r, st);
          hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(kBlock), 0, st, n, -1.0, r, 0.0, r, r);
          h->capture = cap;
          precond(h, r, z, nullptr, st);
          h->capture = nullptr;
          hipLaunchKernelGGL(k_add_cast, dim3(nblk(n)), dim3(kBlock), 0, st, n, e, cap, h->ls_snap + size_t(t) * n);
          hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(kBlock), 0, st, n, 1.0, e, 1.0, z, e);
          // c_t = |L e_t|^2 in the training precision
          SPMV_F32(d.G, n, d.W, d.rowptr, d.col, d.v32, h->ls_snap + size_t(t) * n, h->ls_y);
          fdot(h, n, h->ls_y, h->ls_y, h->ls_c + t, st);
        }
      }
      h->p.precision = prec;
      h->ls_T = T;
    }
    if (h->ls_T < 1 && o->steps > 0) throw Error(MGM_E_ARG, "learned smoother: no snapshots");
    // training
    if (o->steps > 0) {
      if (!h->ls_loss || o->steps + 1 > h->ls_steps_cap) {
        h->ls_loss = track(h, dalloc<double>(o->steps + 1));
        h->ls_steps_cap = o->steps + 1;
      }
      for (int it = 0; it < o->steps; ++it) train_step(h, true, h->ls_loss + it, float(o->lr), st);
      train_step(h, false, h->ls_loss + o->steps, float(o->lr), st);
      std::vector<double> hist(o->steps + 1);
      HIPCHECK(hipMemcpyAsync(hist.data(), h->ls_loss, sizeof(double) * hist.size(), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      info->loss_first = hist.front();
      info->loss_last = hist.back();
      if (h_loss_hist) std::copy(hist.begin(), hist.end(), h_loss_hist);
    }
    compute_omega(h, st);
    // activation: compare stationary convergence factors from the first start
    if (o->activate == 2) {
      set_active(h, true);
    } else if (o->activate == 1 && o->n_starts > 0) {
      double* e0 = h->vecs + 8 * h->ld;
      hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(n)), dim3(kBlock), 0, st, n, d.perm, d_starts, e0,
                         (double*)nullptr);
      set_active(h, false);
      info->rate_gs = stationary_rate(h, e0, 6, st);
      set_active(h, true);
      info->rate_learned = stationary_rate(h, e0, 6, st);
      set_active(h, info->rate_learned < info->rate_gs);
    } else {
      set_active(h, o->activate == 0 ? false : was_active);
    }
    info->active = h->ls_active ? 1 : 0;
    HIPCHECK(hipStreamSynchronize(st));
  });
}

mgm_status mgm_smoother_params(mgm_handle h, int32_t set, float* h_params, int64_t* len) {
  if (!h || !len) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    if (!h->ls_params) throw Error(MGM_E_ARG, "learned smoother not prepared (call mgm_train_smoother first)");
    const int64_t np = mlp_param_count(h->ls_nin, h->ls_s);
    if (!h_params) {
      *len = np;
      return;
    }
    if (*len < np) throw Error(MGM_E_ARG, "parameter buffer too small");
    if (set) {
      HIPCHECK(hipMemcpy(h->ls_params, h_params, np * sizeof(float), hipMemcpyHostToDevice));
      HIPCHECK(hipMemset(h->ls_m, 0, np * sizeof(float)));
      HIPCHECK(hipMemset(h->ls_v, 0, np * sizeof(float)));
      h->ls_adam_t = 0;
      compute_omega(h, nullptr);
      HIPCHECK(hipDeviceSynchronize());
    } else {
      HIPCHECK(hipMemcpy(h_params, h->ls_params, np * sizeof(float), hipMemcpyDeviceToHost));
    }
    *len = np;
  });
}

mgm_status mgm_smoother_grad(mgm_handle h, float* h_grad, double* loss, void* stream) {
  if (!h || !loss) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!h->ls_params || h->ls_T < 1) throw Error(MGM_E_ARG, "learned smoother has no snapshots");
    ensure_ws(h, 1);
    if (!h->ls_loss) {
      h->ls_loss = track(h, dalloc<double>(2));
      h->ls_steps_cap = 2;
    }
    train_step(h, false, h->ls_loss, 0.0f, st);
    const int64_t np = mlp_param_count(h->ls_nin, h->ls_s);
    if (h_grad) HIPCHECK(hipMemcpyAsync(h_grad, h->ls_grad, np * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(loss, h->ls_loss, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
  });
}

mgm_status mgm_set_smoother(mgm_handle h, int32_t learned) {
  if (!h) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    if (learned && !h->ls_om64) throw Error(MGM_E_ARG, "learned smoother not trained");
    set_active(h, learned != 0);
  });
}

}  // extern "C"
