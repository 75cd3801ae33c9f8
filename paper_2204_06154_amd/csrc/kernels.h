// HIP kernels of the MGM solve phase for gfx950 (CDNA4, wave64).
//
// Sparse operators are stored row-major (CSR; the fine level has a fixed row
// width W = stencil size, so its row pointer is implicit). A group of G
// consecutive lanes of a wavefront owns one row: lane t reads entries t,
// t+G, ... so a wavefront reads 64/G consecutive rows as one contiguous
// stream, and the group's partial sums are combined with cross-lane
// shuffles. Operator values are stored as V (double, float or _Float16 with
// one float scale per row) and accumulated in S (double or float).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

namespace mgm {
namespace {  // kernels have internal linkage: each translation unit owns its copies

constexpr int kBlock = 256;

// Lane exchange inside one DPP row of 16 lanes (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, 0xF, 0xF, false));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, 0xF, 0xF, false));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within each 8
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within each 16

// Sum over each aligned group of G consecutive lanes (G = 1, 2, 4, 8, 16);
// every lane of the group gets the same bits. All lanes of a group must be
// active. Each stage adds two partial sums over disjoint lane sets.
template <int G, typename S>
__device__ __forceinline__ S group_sum(S v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
  if constexpr (G >= 16) v += dpp_mov<kDppMirror>(v);
  if constexpr (G >= 8) v += dpp_mov<kDppHalfMirror>(v);
  if constexpr (G >= 4) v += dpp_mov<kDppXor2>(v);
  if constexpr (G >= 2) v += dpp_mov<kDppXor1>(v);
  return v;
}

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

// Patch-blocked Gauss-Seidel: one workgroup sweeps one patch (<= kPatch rows)
// of the current patch colour, kPatchG consecutive lanes per row. Patches of
// one colour never couple, so the values outside the patch ("halo") are
// constant during the launch: the lanes of a row fold its halo entries into
// the right-hand side once, keep the in-patch entries (value, local column)
// in registers, and the patch values live in LDS. The local colours are then
// visited in order (reverse for a backward sweep), one barrier each: rows of
// one local colour never couple, so this is sequential GS in the order
// (patch colour, patch, local colour).
// With zero_guess the sweep starts from u = 0 without reading u: rows of patch
// colours visited earlier in this sweep hold their new values, all others are
// taken as zero (so no separate clearing pass is needed).
// Operator storage per patch slot: ELL with the level's width nw * kPatchG
// and a fixed stride of `block` rows, entry i*kPatchG + g of local row t at
// (slot * block * nw + i * block + t) * kPatchG + g, so the lanes of a
// workgroup read consecutive addresses and the entry loads depend on no other
// load; padding entries have value zero and a valid column.
constexpr int kPatch = 256;
constexpr int kPatchG = 4;
template <typename V, typename S, int WL, bool SCALED, bool BORDER>
__global__ __launch_bounds__(kPatch * kPatchG) void k_gs_patch(
    int slot0, int reverse, int zero_guess, int nw, int block, const int32_t* __restrict__ pstart,
    const int32_t* __restrict__ pncl, const int32_t* __restrict__ lcol,
    const V* __restrict__ pval, const int32_t* __restrict__ pcol, const float* __restrict__ scale,
    const S* __restrict__ dinv, const S* __restrict__ f, S* u, const S* __restrict__ b,
    const double* __restrict__ lam) {
  __shared__ S ul[kPatch];
  const int slot = slot0 + blockIdx.x;
  const int t = threadIdx.x / kPatchG;
  const int g = threadIdx.x % kPatchG;
  const bool slot_row = t < block;
  // entry loads first: their addresses need no other load
  const int64_t base = (int64_t(slot) * block * nw + t) * kPatchG + g;
  int cc[WL];
  S iv[WL];
#pragma unroll
  for (int i = 0; i < WL; ++i) {
    const int ii = i < nw ? i : nw - 1;  // chunks >= nw: re-read the last one, zeroed below
    const int64_t e = base + int64_t(ii) * block * kPatchG;
    cc[i] = slot_row ? pcol[e] : 0;
    iv[i] = (slot_row && i < nw) ? S(pval[e]) : S(0);
  }
  const int r0 = pstart[slot];
  const int nr = pstart[slot + 1] - r0;
  const int ncl = pncl[slot];
  // rows [upd_lo, upd_hi) hold current values (all rows unless zero_guess)
  int upd_lo = 0, upd_hi = INT_MAX;
  if (zero_guess) {
    if (reverse) upd_lo = pstart[slot0 + gridDim.x];
    else upd_hi = pstart[slot0];
  }
  const bool act = t < nr;
  const int row = r0 + t;
  int ic[WL];
  S rhs = S(0), di = S(0), sc = S(1), uown = S(0);
  int myc = -1;
  if (act) {
    uown = zero_guess ? S(0) : u[row];
    myc = lcol[row];
    di = dinv[row];
    rhs = f[row];
    if (SCALED) sc = S(scale[row]);
    if (BORDER) rhs -= b[row] * S(*lam);
    S halo = S(0);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
      const bool live = i < nw;
      const bool in = live && unsigned(cc[i] - r0) < unsigned(nr);
      const bool cur = cc[i] >= upd_lo && cc[i] < upd_hi;
      const S uv = (live && !in && cur) ? u[cc[i]] : S(0);
      halo += iv[i] * uv;
      ic[i] = in ? cc[i] - r0 : t;
      iv[i] = in ? iv[i] : S(0);
    }
    halo = group_sum<kPatchG>(halo);
    rhs -= sc * halo;
    if (g == 0) ul[t] = uown;
  }
  __syncthreads();
  // Each row keeps its own value in a register (only that row writes it).
  for (int step = 0; step < ncl; ++step) {
    const int c = reverse ? ncl - 1 - step : step;
    if (myc == c) {  // all lanes of a row agree
      S a0 = S(0), a1 = S(0), a2 = S(0), a3 = S(0);
#pragma unroll
      for (int i = 0; i < WL; i += 4) {
        a0 += iv[i] * ul[ic[i]];
        a1 += iv[i + 1] * ul[ic[i + 1]];
        a2 += iv[i + 2] * ul[ic[i + 2]];
        a3 += iv[i + 3] * ul[ic[i + 3]];
      }
      const S acc = group_sum<kPatchG>((a0 + a1) + (a2 + a3));
      uown = uown + (rhs - sc * acc) * di;
      if (g == 0) ul[t] = uown;
    }
    __syncthreads();
  }
  if (act && g == 0) u[row] = uown;
}

// res = f - A u over all rows; with BDOT also per-block partial sums of b.u
// (written to partial[blockIdx.x], fixed order, deterministic).
template <typename V, typename S, int G, bool SCALED, bool BDOT>
__global__ __launch_bounds__(kBlock) void k_residual(int n, int W, const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col, const V* __restrict__ val,
                                                     const float* __restrict__ scale, const S* __restrict__ f,
                                                     const S* __restrict__ u, S* __restrict__ res,
                                                     const S* __restrict__ b, double* __restrict__ partial) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int row = gid / G;
  const int lane = gid % G;
  double bu = 0.0;
  if (row < n) {
    S acc = row_dot<V, S, G, SCALED>(row, lane, W, rowptr, col, val, scale, u);
    if (lane == 0) {
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
template <typename V, typename S>
__global__ __launch_bounds__(kBlock) void k_interp_add(int n, int m, const int32_t* __restrict__ pcol,
                                                       const V* __restrict__ pval, const S* __restrict__ ec,
                                                       S* __restrict__ e) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  S acc = S(0);
  for (int t = 0; t < m; ++t) acc += S(pval[i * m + t]) * ec[pcol[i * m + t]];
  e[i] += acc;
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
constexpr int kMaxDots = 200;  // vectors of one dot launch (the FGMRES restart limit)

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
