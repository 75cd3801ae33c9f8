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

// The MLP's per-node products on the FP32 matrix cores: each wavefront takes
// 16 nodes and runs every layer as v_mfma_f32_16x16x4f32 tiles (16 nodes x
// 16 outputs, four inputs per step; lane 16k + i supplies input k of node i
// and weight row k for output i; accumulator register v of lane 16g + c is
// node 4g + v, output c). The weights are read through the caches (the same
// few tens of KB for every wavefront); each layer's output goes through a
// 16 x 65 LDS tile ([h; 1], the 1 multiplying the next layer's bias row) to
// become the next layer's input, and from there, row by row, to the
// activation arrays the gradient needs.
typedef float mlp_f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMlpWaves = 4;
constexpr int kMlpNodes = 16 * kMlpWaves;  // nodes per workgroup
constexpr int kActStride = kHid + 1;        // [h; 1]

__device__ __forceinline__ void mlp_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// rows of a wavefront's 16 x 65 tile to H (N x 65, row-major), nodes < n
__device__ __forceinline__ void mlp_store_tile(const float* tile, float* __restrict__ H, int node0, int n, int lane) {
  for (int r = 0; r < 16 && node0 + r < n; ++r) {
    float* hr = H + size_t(node0 + r) * kActStride;
    hr[lane] = tile[r * kActStride + lane];
    if (lane == 0) hr[kHid] = 1.0f;
  }
}

// relu(acc) of four 16 x 16 output tiles into the wavefront's tile, with the
// ones column
__device__ __forceinline__ void mlp_relu_to_tile(const mlp_f32x4 (&acc)[4], float* tile, int ki, int li, int lane) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) tile[(4 * ki + v) * kActStride + 16 * t + li] = fmaxf(acc[t][v], 0.0f);
  if (lane < 16) tile[lane * kActStride + kHid] = 1.0f;
}

// MLP forward for every node: o = W3 relu(W2 relu(W1 x + b1) + b2) + b3
// (the bias rows multiply the trailing 1 of x and of each [h; 1]) and, for
// training (H1 non-null), the augmented activations [h; 1] (N x 65 each).
// Weights: W1 (nin+1) x 64, W2 65 x 64, W3 65 x s, row-major, consecutive.
__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_forward(int n, int nin, int s, const float* __restrict__ X,
                                                               const float* __restrict__ params, float* __restrict__ O,
                                                               float* __restrict__ H1, float* __restrict__ H2) {
  __shared__ float act[kMlpWaves][16 * kActStride];
  const int wave = int(threadIdx.x) / 64, lane = int(threadIdx.x) % 64;
  const int ki = lane / 16, li = lane % 16;
  const int node0 = (int(blockIdx.x) * kMlpWaves + wave) * 16;
  if (node0 >= n) return;  // no workgroup barrier follows
  const int ka = nin + 1;
  const float* W1 = params;
  const float* W2 = W1 + size_t(ka) * kHid;
  const float* W3 = W2 + size_t(kActStride) * kHid;
  float* tile = act[wave];
  const bool arow = node0 + li < n;
  const float* xr = X + size_t(arow ? node0 + li : node0) * ka;
  mlp_f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = mlp_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < ka; k0 += 4) {
    const int k = k0 + ki;
    const bool kin = k < ka;
    const float a = (arow && kin) ? xr[k] : 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float b = kin ? W1[size_t(k) * kHid + 16 * t + li] : 0.0f;
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
    }
  }
  mlp_relu_to_tile(acc, tile, ki, li, lane);
  mlp_wave_sync();
  if (H1) mlp_store_tile(tile, H1, node0, n, lane);
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = mlp_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < kActStride; k0 += 4) {
    const int k = k0 + ki;
    const bool kin = k < kActStride;
    const float a = kin ? tile[li * kActStride + k] : 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float b = kin ? W2[size_t(k) * kHid + 16 * t + li] : 0.0f;
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
    }
  }
  mlp_wave_sync();  // every read of the layer-1 tile precedes its overwrite
  mlp_relu_to_tile(acc, tile, ki, li, lane);
  mlp_wave_sync();
  if (H2) mlp_store_tile(tile, H2, node0, n, lane);
  mlp_f32x4 o = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < kActStride; k0 += 4) {
    const int k = k0 + ki;
    const bool kin = k < kActStride;
    const float a = kin ? tile[li * kActStride + k] : 0.0f;
    const float b = (kin && li < s) ? W3[size_t(k) * s + li] : 0.0f;
    o = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, o, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int node = node0 + 4 * ki + v;
    if (node < n && li < s) O[size_t(node) * s + li] = o[v];
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
// dH2 = relu'(h2) (W3 dO); dH1 = relu'(h1) (W2 dH2) (the bias rows of W3 and
// W2 take no part). Same tiling as the forward pass: dO, then dH2, pass
// through the wavefront's LDS tile to become the next product's input.
__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_backward(int n, int nin, int s, const float* __restrict__ params,
                                                                const float* __restrict__ O, const float* __restrict__ domega,
                                                                const double* __restrict__ wcheb, const float* __restrict__ H1,
                                                                const float* __restrict__ H2, float* __restrict__ dO,
                                                                float* __restrict__ dH1, float* __restrict__ dH2) {
  __shared__ float act[kMlpWaves][16 * kActStride];
  const int wave = int(threadIdx.x) / 64, lane = int(threadIdx.x) % 64;
  const int ki = lane / 16, li = lane % 16;
  const int node0 = (int(blockIdx.x) * kMlpWaves + wave) * 16;
  if (node0 >= n) return;  // no workgroup barrier follows
  const float* W2 = params + size_t(nin + 1) * kHid;
  const float* W3 = W2 + size_t(kActStride) * kHid;
  float* tile = act[wave];
  // dO of the wavefront's 16 nodes (zero past n) into the tile
  for (int idx = lane; idx < 16 * s; idx += 64) {
    const int r = idx / s, q = idx % s;
    const int node = node0 + r;
    float d = 0.0f;
    if (node < n) {
      const float th = tanhf(O[size_t(node) * s + q]);
      d = domega[size_t(q) * n + node] * float(wcheb[q]) * 0.5f * (1.0f - th * th);
      dO[size_t(node) * s + q] = d;
    }
    tile[r * kActStride + q] = d;
  }
  mlp_wave_sync();
  // dH2 = relu'(h2) (dO W3^T): inputs q < s, weights W3[j][q]
  mlp_f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = mlp_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < s; k0 += 4) {
    const int q = k0 + ki;
    const bool kin = q < s;
    const float a = kin ? tile[li * kActStride + q] : 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float b = kin ? W3[size_t(16 * t + li) * s + q] : 0.0f;
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
    }
  }
  mlp_wave_sync();  // every read of dO precedes the overwrite
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int node = node0 + 4 * ki + v, j = 16 * t + li;
      float g = 0.0f;
      if (node < n) {
        g = H2[size_t(node) * kActStride + j] > 0.0f ? acc[t][v] : 0.0f;
        dH2[size_t(node) * kHid + j] = g;
      }
      tile[(4 * ki + v) * kActStride + j] = g;
    }
  mlp_wave_sync();
  // dH1 = relu'(h1) (dH2 W2^T): inputs o < 64, weights W2[k][o]
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = mlp_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < kHid; k0 += 4) {
    const int o = k0 + ki;
    const float a = tile[li * kActStride + o];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float b = W2[size_t(16 * t + li) * kHid + o];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int node = node0 + 4 * ki + v, k = 16 * t + li;
      if (node < n) dH1[size_t(node) * kHid + k] = H1[size_t(node) * kActStride + k] > 0.0f ? acc[t][v] : 0.0f;
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
  // The next tile's loads are issued into registers before the current
  // tile's products, so that their latency overlaps the matrix-core work;
  // rows past the chunk's end load as zeros.
  constexpr int kThreads = 64 * kAtbWaves;
  constexpr int kPerA = (kAtbTile * kAtbMaxK + kThreads - 1) / kThreads;
  constexpr int kPerB = (kAtbTile * 16 * NBJ + kThreads - 1) / kThreads;
  float ra[kPerA], rb[kPerB];
  auto fetch = [&](int t0) {
    const int nt = min(kAtbTile, n1 - t0);
#pragma unroll
    for (int i = 0; i < kPerA; ++i) {
      const int e = int(threadIdx.x) + i * kThreads;
      ra[i] = e < nt * ka ? A[size_t(t0) * ka + e] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < kPerB; ++i) {
      const int e = int(threadIdx.x) + i * kThreads;
      rb[i] = e < nt * kb ? B[size_t(t0) * kb + e] : 0.0f;
    }
  };
  if (n0 < n1) fetch(n0);
  for (int t0 = n0; t0 < n1; t0 += kAtbTile) {
#pragma unroll
    for (int i = 0; i < kPerA; ++i) {
      const int e = int(threadIdx.x) + i * kThreads;
      if (e < kAtbTile * ka) sa[e] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < kPerB; ++i) {
      const int e = int(threadIdx.x) + i * kThreads;
      if (e < kAtbTile * kb) sb[e] = rb[i];
    }
    __syncthreads();
    if (t0 + kAtbTile < n1) fetch(t0 + kAtbTile);
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

// Sum of the per-block partials, deterministic in two stages (FP64):
// stage 1, per entry e and group y of kColGroup consecutive blocks,
// part2[y][e] = sum over the group's blocks in order; stage 2, out[e] = the
// sum of part2[.][e] over the groups in order.
constexpr int kColGroup = 16;
__global__ __launch_bounds__(kBlock) void k_reduce_cols_group(int nblocks, int nc, const float* __restrict__ partial,
                                                              double* __restrict__ part2) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= nc) return;
  const int b0 = int(blockIdx.y) * kColGroup, b1 = min(nblocks, b0 + kColGroup);
  double acc = 0.0;
  for (int b = b0; b < b1; ++b) acc += double(partial[size_t(b) * nc + e]);
  part2[size_t(blockIdx.y) * nc + e] = acc;
}
__global__ __launch_bounds__(kBlock) void k_reduce_cols(int ngroups, int nc, const double* __restrict__ part2,
                                                        float* __restrict__ out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= nc) return;
  double acc = 0.0;
  for (int y = 0; y < ngroups; ++y) acc += part2[size_t(y) * nc + e];
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
