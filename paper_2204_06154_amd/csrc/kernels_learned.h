// HIP kernels of the learned per-node Chebyshev smoother (fine level).
//
// Inference: s Richardson steps e <- e + omega_q D^-1 (f - L e) with per-node
// step weights omega. Training (homogeneous problem, FP32): forward steps
// z_q = D^-1 L e_{q-1}, e_q = e_{q-1} - omega_q z_q; loss |L e_s|^2/|L e_0|^2;
// adjoint g_{q-1} = g_q - L^T D^-1 (omega_q g_q), dLoss/domega_q = -g_q z_q;
// MLP (3n -> 64 -> 64 -> s, ReLU) forward/backward with one thread per node and
// the weights staged in LDS; weight gradients as deterministic two-stage
// reductions A^T B over the nodes; Adam.
//
// Parameter layout (FP32, row-major, the bias as the last row of each layer):
//   W1aug (nin+1) x 64 | W2aug 65 x 64 | W3aug 65 x s.
#pragma once

#include "kernels.h"

namespace mgm {
namespace {  // kernels have internal linkage: each translation unit owns its copies

constexpr int kHid = 64;

__host__ __device__ inline int mlp_param_count(int nin, int s) { return (nin + 1) * kHid + (kHid + 1) * kHid + (kHid + 1) * s; }

// e_out = e_in + omega * dinv * (f - A e_in)   (one Richardson step); with
// BORDER the bordered system's multiplier is held fixed at *lam:
// e_out = e_in + omega * dinv * (f - (A e_in + b *lam))
template <typename V, typename S, int G, bool SCALED, bool BORDER>
__global__ __launch_bounds__(kBlock) void k_richardson(int n, int W, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, const V* __restrict__ val,
                                                       const float* __restrict__ scale, const S* __restrict__ dinv,
                                                       const S* __restrict__ omega, const S* __restrict__ f,
                                                       const S* __restrict__ ein, S* __restrict__ eout,
                                                       const S* __restrict__ b, const double* __restrict__ lam) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int row = gid / G;
  const int lane = gid % G;
  if (row >= n) return;
  const S fr = f[row], di = dinv[row], om = omega[row], er = ein[row];
  S acc = row_dot<V, S, G, SCALED>(row, lane, W, rowptr, col, val, scale, ein);
  if (BORDER) acc += b[row] * S(*lam);
  if (lane == 0) eout[row] = er + om * di * (fr - acc);
}

// First Richardson step from e = 0: e = omega * dinv * f (same association
// as k_richardson with e_in = 0).
template <typename S>
__global__ __launch_bounds__(kBlock) void k_scale_start(int n, const S* __restrict__ omega, const S* __restrict__ dinv,
                                                        const S* __restrict__ f, S* __restrict__ e) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) e[i] = omega[i] * dinv[i] * f[i];
}

// training forward step: z = dinv * (A e_in); e_out = e_in - omega * z (FP32)
template <int G>
__global__ __launch_bounds__(kBlock) void k_train_step(int n, int W, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, const float* __restrict__ val,
                                                       const float* __restrict__ dinv, const float* __restrict__ omega,
                                                       const float* __restrict__ ein, float* __restrict__ eout,
                                                       float* __restrict__ z) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int row = gid / G;
  const int lane = gid % G;
  if (row >= n) return;
  const float di = dinv[row], om = omega[row], er = ein[row];
  float acc = row_dot<float, float, G, false>(row, lane, W, rowptr, col, val, nullptr, ein);
  if (lane == 0) {
    const float zz = di * acc;
    z[row] = zz;
    eout[row] = er - om * zz;
  }
}

// y = x - A t  (adjoint step with A = L^T; x may alias y only if A has no
// reads of y, which holds: t is a separate buffer)
template <int G>
__global__ __launch_bounds__(kBlock) void k_xmAt(int n, int W, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const float* __restrict__ val,
                                                 const float* __restrict__ x, const float* __restrict__ t,
                                                 float* __restrict__ y) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int row = gid / G;
  const int lane = gid % G;
  if (row >= n) return;
  const float xr = x[row];
  float acc = row_dot<float, float, G, false>(row, lane, W, rowptr, col, val, nullptr, t);
  if (lane == 0) y[row] = xr - acc;
}

// domega_q += -g * z_q ; t = dinv * omega_q * g
__global__ __launch_bounds__(kBlock) void k_adj_accum(int n, const float* __restrict__ g, const float* __restrict__ z,
                                                      const float* __restrict__ dinv, const float* __restrict__ omega,
                                                      float* __restrict__ domega, float* __restrict__ t) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  domega[i] -= gi * z[i];
  t[i] = dinv[i] * omega[i] * gi;
}

// y *= factor[0] (device scalar, FP64)
__global__ __launch_bounds__(kBlock) void k_scale_dev(int n, const double* __restrict__ factor, float* __restrict__ y) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = float(double(y[i]) * factor[0]);
}

// loss += yy / ct * invT ;  (device scalars)
__global__ void k_loss_acc(const double* __restrict__ yy, const double* __restrict__ ct, double invT,
                           double* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) loss[0] += yy[0] / ct[0] * invT;
}

// y *= mult / ct  (FP32 vector, FP64 device scalar)
__global__ __launch_bounds__(kBlock) void k_scale_ct(int n, const double* __restrict__ ct, double mult,
                                                     float* __restrict__ y) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = float(double(y[i]) * (mult / ct[0]));
}

// out = float(a + b)  (snapshot = iterate + captured correction)
__global__ __launch_bounds__(kBlock) void k_add_cast(int n, const double* __restrict__ a, const double* __restrict__ b,
                                                     float* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = float(a[i] + b[i]);
}

// factor = num / den  (device scalars)
__global__ void k_ratio(const double* __restrict__ num, const double* __restrict__ den, double mult,
                        double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = mult * num[0] / den[0];
}

// per-block partial sums of x.y (FP32 vectors, FP64 accumulation)
__global__ __launch_bounds__(kBlock) void k_fdot_partial(int n, const float* __restrict__ x, const float* __restrict__ y,
                                                         double* __restrict__ partial) {
  const int nb = gridDim.x;
  const int64_t chunk = (int64_t(n) + nb - 1) / nb;
  const int64_t b0 = chunk * blockIdx.x;
  const int64_t b1 = min(int64_t(n), b0 + chunk);
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) acc += double(x[i]) * double(y[i]);
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// MLP forward for every node: o = W3 relu(W2 relu(W1 x + b1) + b2) + b3 and,
// for training, the augmented activations [h; 1] (N x 65 each).
__global__ __launch_bounds__(kBlock) void k_mlp_forward(int n, int nin, int s, const float* __restrict__ X,
                                                        const float* __restrict__ params, float* __restrict__ O,
                                                        float* __restrict__ H1, float* __restrict__ H2) {
  extern __shared__ float wsh[];
  const int np = mlp_param_count(nin, s);
  for (int k = threadIdx.x; k < np; k += kBlock) wsh[k] = params[k];
  __syncthreads();
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float* W1 = wsh;
  const float* W2 = W1 + (nin + 1) * kHid;
  const float* W3 = W2 + (kHid + 1) * kHid;
  const float* x = X + size_t(i) * (nin + 1);
  float h1[kHid];
#pragma unroll
  for (int o = 0; o < kHid; ++o) h1[o] = W1[nin * kHid + o];
  for (int k = 0; k < nin; ++k) {
    const float xk = x[k];
#pragma unroll
    for (int o = 0; o < kHid; ++o) h1[o] += xk * W1[k * kHid + o];
  }
#pragma unroll
  for (int o = 0; o < kHid; ++o) h1[o] = fmaxf(h1[o], 0.0f);
  float h2[kHid];
#pragma unroll
  for (int o = 0; o < kHid; ++o) h2[o] = W2[kHid * kHid + o];
#pragma unroll
  for (int k = 0; k < kHid; ++k) {
#pragma unroll
    for (int o = 0; o < kHid; ++o) h2[o] += h1[k] * W2[k * kHid + o];
  }
#pragma unroll
  for (int o = 0; o < kHid; ++o) h2[o] = fmaxf(h2[o], 0.0f);
  for (int q = 0; q < s; ++q) {
    float acc = W3[kHid * s + q];
#pragma unroll
    for (int k = 0; k < kHid; ++k) acc += h2[k] * W3[k * s + q];
    O[size_t(i) * s + q] = acc;
  }
  if (H1) {
#pragma unroll
    for (int o = 0; o < kHid; ++o) {
      H1[size_t(i) * (kHid + 1) + o] = h1[o];
      H2[size_t(i) * (kHid + 1) + o] = h2[o];
    }
    H1[size_t(i) * (kHid + 1) + kHid] = 1.0f;
    H2[size_t(i) * (kHid + 1) + kHid] = 1.0f;
  }
}

// omega[q][i] = wcheb_q (1 + 0.5 tanh(O[i][q])) in the smoother's precision
template <typename S>
__global__ __launch_bounds__(kBlock) void k_omega(int n, int s, const float* __restrict__ O,
                                                  const double* __restrict__ wcheb, S* __restrict__ omega) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < s; ++q) omega[size_t(q) * n + i] = S(wcheb[q] * (1.0 + 0.5 * tanh(double(O[size_t(i) * s + q]))));
}

// MLP backward per node: dO = domega * wcheb * 0.5 (1 - tanh^2 o);
// dH2 = relu'(h2) (W3 dO); dH1 = relu'(h1) (W2 dH2).
__global__ __launch_bounds__(kBlock) void k_mlp_backward(int n, int nin, int s, const float* __restrict__ params,
                                                         const float* __restrict__ O, const float* __restrict__ domega,
                                                         const double* __restrict__ wcheb, const float* __restrict__ H1,
                                                         const float* __restrict__ H2, float* __restrict__ dO,
                                                         float* __restrict__ dH1, float* __restrict__ dH2) {
  extern __shared__ float wsh[];
  const int np = mlp_param_count(nin, s);
  for (int k = threadIdx.x; k < np; k += kBlock) wsh[k] = params[k];
  __syncthreads();
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float* W2 = wsh + (nin + 1) * kHid;
  const float* W3 = W2 + (kHid + 1) * kHid;
  float dq[8];
  for (int q = 0; q < s; ++q) {
    const float th = tanhf(O[size_t(i) * s + q]);
    dq[q] = domega[size_t(q) * n + i] * float(wcheb[q]) * 0.5f * (1.0f - th * th);
    dO[size_t(i) * s + q] = dq[q];
  }
  float g2[kHid];
#pragma unroll
  for (int k = 0; k < kHid; ++k) {
    float acc = 0.0f;
    for (int q = 0; q < s; ++q) acc += W3[k * s + q] * dq[q];
    g2[k] = H2[size_t(i) * (kHid + 1) + k] > 0.0f ? acc : 0.0f;
    dH2[size_t(i) * kHid + k] = g2[k];
  }
#pragma unroll 4
  for (int k = 0; k < kHid; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int o = 0; o < kHid; ++o) acc += W2[k * kHid + o] * g2[o];
    dH1[size_t(i) * kHid + k] = H1[size_t(i) * (kHid + 1) + k] > 0.0f ? acc : 0.0f;
  }
}

// C_partial[blk] = sum over the block's chunk of kAtbChunk nodes of
// A[i]^T B[i] (A: N x ka, B: N x kb, row-major FP32; C: ka x kb, row-major),
// a dense contraction over the nodes, on the FP32 matrix cores: C is cut into
// 16 x 16 tiles, wave w owns the tile rows w, w + kAtbWaves, ... and all NBJ
// tile columns (kb <= 16 NBJ), and each v_mfma_f32_16x16x4f32 takes four
// nodes as its K dimension (lane 16k + i supplies A[node k][16 bi + i] and
// B[node k][16 bj + i]; accumulator register v of lane 16g + c holds
// C[16 bi + 4g + v][16 bj + c]). Tiles of kAtbTile nodes of A and B are staged
// in LDS with coalesced loads, zero past the chunk's end and outside C. The
// summation order is fixed, so the result is deterministic.
typedef float atb_f32x4 __attribute__((ext_vector_type(4)));
constexpr int kAtbChunk = 512;
constexpr int kAtbTile = 32;
constexpr int kAtbMaxK = 200;  // columns of A at most
constexpr int kAtbWaves = 4;
constexpr int kAtbRowsPerWave = ((kAtbMaxK + 15) / 16 + kAtbWaves - 1) / kAtbWaves;
template <int NBJ>
__global__ __launch_bounds__(64 * kAtbWaves) void k_atb_partial(int n, int ka, int kb, const float* __restrict__ A,
                                                               const float* __restrict__ B, float* __restrict__ partial) {
  __shared__ float sa[kAtbTile * kAtbMaxK];
  __shared__ float sb[kAtbTile * 16 * NBJ];
  const int wave = int(threadIdx.x) / 64, lane = int(threadIdx.x) % 64;
  const int ki = lane / 16, li = lane % 16;
  const int n0 = int(blockIdx.x) * kAtbChunk;
  const int n1 = min(n, n0 + kAtbChunk);
  const int nbi = (ka + 15) / 16;
  atb_f32x4 acc[kAtbRowsPerWave][NBJ];
#pragma unroll
  for (int r = 0; r < kAtbRowsPerWave; ++r)
#pragma unroll
    for (int bj = 0; bj < NBJ; ++bj) acc[r][bj] = atb_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int t0 = n0; t0 < n1; t0 += kAtbTile) {
    const int nt = min(kAtbTile, n1 - t0);
    for (int e = int(threadIdx.x); e < kAtbTile * ka; e += int(blockDim.x))
      sa[e] = e < nt * ka ? A[size_t(t0) * ka + e] : 0.0f;
    for (int e = int(threadIdx.x); e < kAtbTile * kb; e += int(blockDim.x))
      sb[e] = e < nt * kb ? B[size_t(t0) * kb + e] : 0.0f;
    __syncthreads();
#pragma unroll 2
    for (int k0 = 0; k0 < kAtbTile; k0 += 4) {
      const int node = k0 + ki;
      float bop[NBJ];
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) {
        const int col = bj * 16 + li;
        bop[bj] = col < kb ? sb[node * kb + col] : 0.0f;
      }
#pragma unroll
      for (int r = 0; r < kAtbRowsPerWave; ++r) {
        const int bi = wave + kAtbWaves * r;
        if (bi < nbi) {  // the same for every lane of the wave
          const int row = bi * 16 + li;
          const float aop = row < ka ? sa[node * ka + row] : 0.0f;
#pragma unroll
          for (int bj = 0; bj < NBJ; ++bj)
            acc[r][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop[bj], acc[r][bj], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  float* out = partial + size_t(blockIdx.x) * ka * kb;
#pragma unroll
  for (int r = 0; r < kAtbRowsPerWave; ++r) {
    const int bi = wave + kAtbWaves * r;
    if (bi >= nbi) continue;
#pragma unroll
    for (int bj = 0; bj < NBJ; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = bi * 16 + 4 * ki + v, jj = bj * 16 + li;
        if (i < ka && jj < kb) out[size_t(i) * kb + jj] = acc[r][bj][v];
      }
  }
}

// out[e] = sum_blk partial[blk][e] in block order (FP64 accumulation)
__global__ __launch_bounds__(kBlock) void k_reduce_cols(int nblocks, int nc, const float* __restrict__ partial,
                                                        float* __restrict__ out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= nc) return;
  double acc = 0.0;
  for (int b = 0; b < nblocks; ++b) acc += double(partial[size_t(b) * nc + e]);
  out[e] = float(acc);
}

// Adam (Kingma & Ba): m, v moments; bias corrections c1 = 1-b1^t, c2 = 1-b2^t
__global__ __launch_bounds__(kBlock) void k_adam(int np, float* __restrict__ p, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                 float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= np) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// power-iteration start v(pos) = u(perm[pos]) - 1/2, u(k) = (splitmix64(k) >> 11) 2^-53
__global__ __launch_bounds__(kBlock) void k_counter_start(int n, const int32_t* __restrict__ perm, double* __restrict__ v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint64_t z = uint64_t(perm ? perm[i] : i) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  v[i] = double(z >> 11) * 0x1.0p-53 - 0.5;
}

// w = dinv * (A v) / sqrt(nrm2)  (power step on the normalised v, FP64)
template <int G>
__global__ __launch_bounds__(kBlock) void k_power_step(int n, int W, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ dinv, const double* __restrict__ nrm2,
                                                       const double* __restrict__ v, double* __restrict__ w) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int row = gid / G;
  const int lane = gid % G;
  if (row >= n) return;
  const double inv = 1.0 / sqrt(nrm2[0]);
  double acc = row_dot<double, double, G, false>(row, lane, W, rowptr, col, val, nullptr, v);
  if (lane == 0) w[row] = dinv[row] * acc * inv;
}

}  // namespace
}  // namespace mgm
