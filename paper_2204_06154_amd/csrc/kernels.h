// HIP kernels of the MGM solve phase for gfx950 (CDNA4, wave64).
//
// Sparse operators are stored row-major (CSR; the fine level has a fixed row
// width W = stencil size, so its row pointer is implicit). A group of G
// consecutive lanes of a wavefront owns one row: lane t reads entries t,
// t+G, ... so a wavefront reads 64/G consecutive rows as one contiguous
// stream, and the group's partial sums are combined with DPP lane moves
// (lane_ops.h). The patch-blocked smoother kernel is in gs_patch.h. Operator values are stored as V (double, float or _Float16 with
// one float scale per row) and accumulated in S (double or float).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include "lane_ops.h"

namespace mgm {
namespace {  // kernels have internal linkage: each translation unit owns its copies

constexpr int kBlock = 256;

template <typename V>
__device__ __forceinline__ float to_f(V v) { return float(v); }

// Row operator: sum_k A_ik x_k for the row owned by this lane group.
template <typename V, typename S, int G, bool SCALED>
__device__ __forceinline__ S row_dot(int row, int lane, int W, const int32_t* __restrict__ rowptr,
                                     const int32_t* __restrict__ col, const V* __restrict__ val,
                                     const float* __restrict__ scale, const S* __restrict__ x) {
  int beg, end;
  if (W > 0) {
    beg = row * W;
    end = beg + W;
  } else {
    beg = rowptr[row];
    end = rowptr[row + 1];
  }
  S acc = S(0);
#pragma unroll 4
  for (int k = beg + lane; k < end; k += G) acc += S(val[k]) * x[col[k]];
  acc = group_sum<G>(acc);
  if (SCALED) acc *= S(scale[row]);
  return acc;
}

// One colour phase of multicolour Gauss-Seidel on rows [r0, r1):
//   u_i += (f_i - sum_k L_ik u_k - b_i lambda) * dinv_i
// Rows of one colour are not coupled, so every row reads only values of
// other colours (and its own old value) while it is written.
template <typename V, typename S, int G, bool SCALED, bool BORDER>
__global__ __launch_bounds__(kBlock) void k_gs_colour(int r0, int r1, int W, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const V* __restrict__ val,
                                                      const float* __restrict__ scale, const S* __restrict__ dinv,
                                                      const S* __restrict__ f, S* u, const S* __restrict__ b,
                                                      const double* __restrict__ lam) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int row = r0 + gid / G;
  const int lane = gid % G;
  if (row >= r1) return;  // whole lane groups exit together
  // issue the row's own loads before the dependent gather chain
  S fr = f[row], di = dinv[row], ui = u[row];
  S bl = S(0);
  if (BORDER) bl = b[row] * S(*lam);
  S acc = row_dot<V, S, G, SCALED>(row, lane, W, rowptr, col, val, scale, u);
  if (lane == 0) u[row] = ui + ((fr - acc) - bl) * di;
}

}  // namespace
}  // namespace mgm

#include "gs_patch.h"

namespace mgm {
namespace {

// res = f - A u (- b lambda when lam is given) over all rows; with BDOT also
// per-block partial sums of b.u
// (written to partial[blockIdx.x], fixed order, deterministic).
template <typename V, typename S, int G, bool SCALED, bool BDOT>
__global__ __launch_bounds__(kBlock) void k_residual(int n, int W, const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col, const V* __restrict__ val,
                                                     const float* __restrict__ scale, const S* __restrict__ f,
                                                     const S* __restrict__ u, S* __restrict__ res,
                                                     const S* __restrict__ b, double* __restrict__ partial,
                                                     const double* __restrict__ lam = nullptr) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int row = gid / G;
  const int lane = gid % G;
  double bu = 0.0;
  if (row < n) {
    S acc = row_dot<V, S, G, SCALED>(row, lane, W, rowptr, col, val, scale, u);
    if (lane == 0) {
      if (lam) acc += b[row] * S(*lam);  // bordered, continuing iterate: f - L u - b lambda
      res[row] = f[row] - acc;
      if (BDOT) bu = double(b[row]) * double(u[row]);
    }
  }
  if (BDOT) {
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = bu;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
  }
}

// y = A x (+ b * lambda when BORDER), all rows.
template <typename V, typename S, int G, bool SCALED, bool BORDER>
__global__ __launch_bounds__(kBlock) void k_spmv(int n, int W, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const V* __restrict__ val,
                                                 const float* __restrict__ scale, const S* __restrict__ x,
                                                 S* __restrict__ y, const S* __restrict__ b,
                                                 const S* __restrict__ lam) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int row = gid / G;
  const int lane = gid % G;
  if (row >= n) return;
  S acc = row_dot<V, S, G, SCALED>(row, lane, W, rowptr, col, val, scale, x);
  if (lane == 0) {
    if (BORDER) acc += b[row] * (*lam);
    y[row] = acc;
  }
}

// Restriction rc = R res (CSR, ~12 entries per row: 4 lanes per row). With
// RHO, block 0 also forms rho_out = rho_in - sum(partial[0..np)) in fixed order.
constexpr int kRestrictG = 4;
template <typename V, typename S, bool RHO>
__global__ __launch_bounds__(kBlock) void k_restrict(int nc, const int32_t* __restrict__ rptr,
                                                     const int32_t* __restrict__ rcol, const V* __restrict__ rval,
                                                     const S* __restrict__ res, S* __restrict__ rc,
                                                     const double* __restrict__ partial, int np,
                                                     const double* __restrict__ rho_in, double* __restrict__ rho_out) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int i = gid / kRestrictG;
  const int lane = gid % kRestrictG;
  if (i < nc) {
    S acc = S(0);
    for (int k = rptr[i] + lane; k < rptr[i + 1]; k += kRestrictG) acc += S(rval[k]) * res[rcol[k]];
    acc = group_sum<kRestrictG>(acc);
    if (lane == 0) rc[i] = acc;
  }
  if (RHO && blockIdx.x == 0) {
    __shared__ double sh[kBlock];
    double s = 0.0;
    for (int t = threadIdx.x; t < np; t += kBlock) s += partial[t];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) *rho_out = *rho_in - sh[0];
  }
}

// Interpolation and correction e += P ec (P: fixed width m, row-major).
// Bordered: the multiplier correction goes up with it, mu_j = mu_{j+1}, or
// mu_j += mu_{j+1} when the level continues from an earlier iterate.
template <typename V, typename S>
__global__ __launch_bounds__(kBlock) void k_interp_add(int n, int m, const int32_t* __restrict__ pcol,
                                                       const V* __restrict__ pval, const S* __restrict__ ec,
                                                       S* __restrict__ e, const double* __restrict__ mu_in = nullptr,
                                                       double* __restrict__ mu_out = nullptr, int accumulate = 0,
                                                       S* __restrict__ out = nullptr) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (mu_out && i == 0) *mu_out = (accumulate ? *mu_out : 0.0) + *mu_in;
  if (i >= n) return;
  S acc = S(0);
  for (int t = 0; t < m; ++t) acc += S(pval[i * m + t]) * ec[pcol[i * m + t]];
  const S v = e[i] + acc;
  if (out) out[i] = v;  // out of place (e left as it was)
  else e[i] = v;
}

// Coarsest solve by the dense FP64 inverse: x = Ainv [rc; rho]; one
// wavefront per output row. Bordered: the last row is the multiplier.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_coarse_gemv(int dim, int np, const double* __restrict__ Ainv,
                                                        const S* __restrict__ rc, const double* __restrict__ rho,
                                                        S* __restrict__ ec, double* __restrict__ mu) {
  const int wave = (blockIdx.x * kBlock + threadIdx.x) / 64;
  const int lane = threadIdx.x % 64;
  if (wave >= dim) return;
  const double* a = Ainv + size_t(wave) * dim;
  double acc = 0.0;
  for (int k = lane; k < np; k += 64) acc += a[k] * double(rc[k]);
  if (dim > np && lane == 0) acc += a[np] * (*rho);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) {
    if (wave < np) ec[wave] = S(acc);
    else *mu = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int n, T* __restrict__ x, T v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = v;
}

// out[pos] = in[perm[pos]] (perm may be null: identity), with conversion.
// With a bordered tail, the scalar in[n] is copied to *tail_out.
template <typename Ti, typename To>
__global__ __launch_bounds__(kBlock) void k_gather(int n, const int32_t* __restrict__ perm, const Ti* __restrict__ in,
                                                   To* __restrict__ out, double* __restrict__ tail_out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = To(in[perm ? perm[i] : i]);
  if (tail_out && i == 0) *tail_out = double(in[n]);
}

// out[perm[pos]] = in[pos] with conversion; bordered tail: out[n] = *tail_in.
template <typename Ti, typename To>
__global__ __launch_bounds__(kBlock) void k_scatter(int n, const int32_t* __restrict__ perm, const Ti* __restrict__ in,
                                                    To* __restrict__ out, const double* __restrict__ tail_in) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[perm ? perm[i] : i] = To(in[i]);
  if (tail_in && i == 0) out[n] = To(*tail_in);
}

// ------------------------------------------------------------------ Krylov
// Deterministic two-stage reductions: stage 1 writes one partial per block
// (grid.y selects the vector), stage 2 sums the partials in block order.
constexpr int kRedBlocks = 512;
// vectors of one dot launch: the FGMRES restart limit (200) plus one, since the
// second projection of the last step also takes |w|^2
constexpr int kMaxDots = 201;

// Fixed-tree sum over the kBlock threads of a block (result in thread 0).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// partial[t * nb + blk] = sum over the block's chunk of V[t][i] * w[i]
__global__ __launch_bounds__(kBlock) void k_mdot_partial(int n, const double* __restrict__ V, int64_t ld,
                                                         const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  const int t = blockIdx.y;
  const int nb = gridDim.x;
  const int64_t chunk = (int64_t(n) + nb - 1) / nb;
  const int64_t b0 = chunk * blockIdx.x;
  const int64_t b1 = min(int64_t(n), b0 + chunk);
  const double* v = V + t * ld;
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) acc += v[i] * w[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[t * nb + blockIdx.x] = s;
}

// out[t] = sum_blk partial[t * nb + blk]; host_out (pinned host memory, may
// be null) receives a copy, so the host needs no separate transfer.
__global__ __launch_bounds__(kBlock) void k_reduce_partials(int k, int nb, const double* __restrict__ partial,
                                                            double* __restrict__ out, double* __restrict__ host_out = nullptr) {
  const int t = blockIdx.x;
  if (t >= k) return;
  __shared__ double sh[kBlock];
  double acc = 0.0;
  // fixed assignment of partials to threads and a fixed tree: deterministic
  for (int i = threadIdx.x; i < nb; i += kBlock) acc += partial[t * nb + i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    out[t] = r;
    if (host_out) host_out[t] = r;
  }
}


// k_reduce_partials for dots over the interior rows [0, nrow) of a bordered
// vector y whose last entry y[nrow] is still held as nc partial sums cpart
// (the operator pass's constraint row): every block sums them in the same
// order (block 0 stores y[nrow]) and adds the border term V[t][nrow] y[nrow]
// to its dot.
__global__ __launch_bounds__(kBlock) void k_reduce_partials_border(int k, int nb, const double* __restrict__ partial,
                                                                   double* __restrict__ out, double* __restrict__ host_out,
                                                                   const double* __restrict__ cpart, int nc,
                                                                   const double* __restrict__ V, int64_t ld, int nrow,
                                                                   double* __restrict__ y) {
  const int t = blockIdx.x;
  if (t >= k) return;
  __shared__ double sh[kBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) acc += partial[t * nb + i];
  const double r = block_sum(acc, sh);
  __syncthreads();
  double cacc = 0.0;
  for (int i = threadIdx.x; i < nc; i += kBlock) cacc += cpart[i];
  const double cy = block_sum(cacc, sh);
  if (threadIdx.x == 0) {
    if (t == 0) y[nrow] = cy;
    const double v = r + V[t * ld + nrow] * cy;
    out[t] = v;
    if (host_out) host_out[t] = v;
  }
}

// w[i] -= sum_{t<k} V[t][i] * h[t]
__global__ __launch_bounds__(kBlock) void k_mupdate(int n, const double* __restrict__ V, int64_t ld, int k,
                                                    const double* __restrict__ h, double* __restrict__ w) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double acc = w[i];
  for (int t = 0; t < k; ++t) acc -= V[t * ld + i] * h[t];
  w[i] = acc;
}

// x[i] += sum_{t<k} Z[t][i] * y[t]
__global__ __launch_bounds__(kBlock) void k_madd(int n, const double* __restrict__ Z, int64_t ld, int k,
                                                 const double* __restrict__ y, double* __restrict__ x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double acc = x[i];
  for (int t = 0; t < k; ++t) acc += Z[t * ld + i] * y[t];
  x[i] = acc;
}

// y = x / sqrt(*nrm2)  (nrm2 = squared norm on device)
__global__ __launch_bounds__(kBlock) void k_normalise(int n, const double* __restrict__ x, const double* __restrict__ nrm2,
                                                      double* __restrict__ y) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double s = sqrt(*nrm2);
  y[i] = s > 0.0 ? x[i] / s : 0.0;
}

// k_normalise that also hands the result to the V-cycle: f0 = S(y) on the
// first nf entries and, bordered, *rho = y[nf] (what the preconditioner's
// input cast would write).
template <typename S>
__global__ __launch_bounds__(kBlock) void k_normalise_cast(int n, const double* __restrict__ x,
                                                           const double* __restrict__ nrm2, double* __restrict__ y,
                                                           S* __restrict__ f0, int nf, double* __restrict__ rho) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double s = sqrt(*nrm2);
  const double v = s > 0.0 ? x[i] / s : 0.0;
  y[i] = v;
  if (i < nf) f0[i] = S(v);
  else if (rho && i == nf) *rho = v;
}

// Second Gram-Schmidt update fused with the normalisation: w -= sum_{t<k}
// V[t] h[t], then w /= s with s^2 = h[k] - sum_{t<k} h[t]^2, where h[k] = |w|^2
// before this update (the updated w is orthogonal to V[0..k), so its squared
// norm is that difference; after the first projection the h[t] are small, so
// it does not cancel). s <= 0 gives w = 0. With f0 given, the result is also
// handed to the V-cycle as in k_normalise_cast. w is updated in place.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_mupdate_normalise(int n, const double* __restrict__ V, int64_t ld, int k,
                                                              const double* __restrict__ h, double* __restrict__ w,
                                                              S* __restrict__ f0, int nf, double* __restrict__ rho) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double acc = w[i];
  double hh = 0.0;
  for (int t = 0; t < k; ++t) {
    acc -= V[t * ld + i] * h[t];
    hh += h[t] * h[t];
  }
  const double s2 = h[k] - hh;
  const double s = s2 > 0.0 ? sqrt(s2) : 0.0;
  const double v = s > 0.0 ? acc / s : 0.0;
  w[i] = v;
  if (f0) {
    if (i < nf) f0[i] = S(v);
    else if (rho && i == nf) *rho = v;
  }
}

// BiCGSTAB updates with the scalars read from device memory (so the host
// need not see them first). sc holds, for the current step k and the
// previous one (slot parity), rho = rhat.r, rv = rhat.v, st = s.t, tt = t.t:
// sc[q * 8 + 0..3] for parity q. alpha = rho / rv, omega = st / tt.
constexpr int kBicgRho = 0, kBicgRv = 1, kBicgSt = 2, kBicgTt = 3;
__device__ __forceinline__ double bicg(const double* sc, int q, int what) { return sc[q * 8 + what]; }

// p = r + beta (p - omega_{k-1} v), beta = (rho_k / rho_{k-1}) (alpha_{k-1} / omega_{k-1})
__global__ __launch_bounds__(kBlock) void k_bicg_p(int n, const double* __restrict__ r, const double* __restrict__ v,
                                                   double* __restrict__ p, const double* __restrict__ sc, int q) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int qo = q ^ 1;
  const double omega = bicg(sc, qo, kBicgSt) / bicg(sc, qo, kBicgTt);
  const double alpha = bicg(sc, qo, kBicgRho) / bicg(sc, qo, kBicgRv);
  const double beta = (bicg(sc, q, kBicgRho) / bicg(sc, qo, kBicgRho)) * (alpha / omega);
  const double t = 1.0 * p[i] + (-omega) * v[i];
  p[i] = 1.0 * r[i] + beta * t;
}

// s = r - alpha_k v
__global__ __launch_bounds__(kBlock) void k_bicg_s(int n, const double* __restrict__ r, const double* __restrict__ v,
                                                   double* __restrict__ s, const double* __restrict__ sc, int q) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double alpha = bicg(sc, q, kBicgRho) / bicg(sc, q, kBicgRv);
  s[i] = 1.0 * r[i] + (-alpha) * v[i];
}

// x += alpha_k phat (+ omega_k shat when shat is given); r = s - omega_k t
__global__ __launch_bounds__(kBlock) void k_bicg_x(int n, const double* __restrict__ phat,
                                                   const double* __restrict__ shat, const double* __restrict__ s,
                                                   const double* __restrict__ t, double* __restrict__ x,
                                                   double* __restrict__ r, const double* __restrict__ sc, int q) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double alpha = bicg(sc, q, kBicgRho) / bicg(sc, q, kBicgRv);
  double xi = 1.0 * x[i] + alpha * phat[i];
  if (shat) {
    const double omega = bicg(sc, q, kBicgSt) / bicg(sc, q, kBicgTt);
    xi = 1.0 * xi + omega * shat[i];
    r[i] = 1.0 * s[i] + (-omega) * t[i];
  }
  x[i] = xi;
}

// z = a*x + b*y (a, b host scalars)
__global__ __launch_bounds__(kBlock) void k_axpby(int n, double a, const double* __restrict__ x, double b,
                                                  const double* __restrict__ y, double* __restrict__ z) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) z[i] = a * x[i] + b * y[i];
}

// r = f - r  (in place on r)
__global__ __launch_bounds__(kBlock) void k_rsub(int n, const double* __restrict__ f, double* __restrict__ r) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) r[i] = f[i] - r[i];
}

}  // namespace
}  // namespace mgm
