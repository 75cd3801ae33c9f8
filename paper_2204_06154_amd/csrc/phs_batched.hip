// Batched RBF-FD stencil weights of the Laplace-Beltrami operator on the GPU.
//
// For every node i: project its stencil onto the tangent plane (Sec. 2.1,
// eq. tp_pts), scale by the stencil radius, and solve the PHS saddle-point
// system of eq. rbf_fd_lap,
//     [A P; P^T 0][c; lambda] = [Lap phi; Lap p],
// A_jk = |xi_j - xi_k|^(2k+1), P_jq = monomials (total degree, then
// descending power of x), Lap r^m = m^2 r^(m-2), Lap p(0) = 2 for x^2, y^2.
//
// One wavefront per system: lane r keeps row r of the augmented matrix
// [M | rhs] in registers (S = n + L <= 64 rows). Gauss-Jordan elimination
// with partial pivoting: at step k the lanes that have not yet been a pivot
// compete for max |a_rk| (wave-wide argmax, ties to the lower lane), the
// pivot row is broadcast with v_readlane, and every other row eliminates
// column k. Afterwards each row holds one diagonal entry and the solution is
// rhs / diag. The column loops are fully unrolled, so every register index
// is a compile-time constant (no scratch).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mgm.h"
#include "host_common.h"

namespace mgm {

// status conversion of the C entry points (defined in device.hip)
extern thread_local std::string g_last_error;
mgm_status guard(const std::function<void()>& f);

namespace {

constexpr int kWaves = 4;  // wavefronts (systems) per block

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Maximum of an unsigned 32-bit value over the 64 lanes of a wavefront, all
// lanes active, by DPP: prefix maxima within each row of 16 lanes (row_shr
// 1, 2, 4, 8), then row_bcast:15 and row_bcast:31 carry the row maxima up to
// lane 63, which is read back. Lanes without a DPP source read 0, the
// identity of an unsigned maximum, so each step can fold into one v_max.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  auto mx = [](int x, int y) { return int(uint32_t(x) > uint32_t(y) ? uint32_t(x) : uint32_t(y)); };
  int t = int(v);
  t = mx(t, __builtin_amdgcn_update_dpp(0, t, 0x111, 0xF, 0xF, true));  // row_shr:1
  t = mx(t, __builtin_amdgcn_update_dpp(0, t, 0x112, 0xF, 0xF, true));  // row_shr:2
  t = mx(t, __builtin_amdgcn_update_dpp(0, t, 0x114, 0xF, 0xF, true));  // row_shr:4
  t = mx(t, __builtin_amdgcn_update_dpp(0, t, 0x118, 0xF, 0xF, true));  // row_shr:8
  t = mx(t, __builtin_amdgcn_update_dpp(0, t, 0x142, 0xA, 0xF, true));  // row_bcast:15 into rows 1, 3
  t = mx(t, __builtin_amdgcn_update_dpp(0, t, 0x143, 0xC, 0xF, true));  // row_bcast:31 into rows 2, 3
  return uint32_t(__builtin_amdgcn_readlane(t, 63));
}

__device__ __forceinline__ double ipow_d(double x, int e) {
  double r = 1.0;
  for (int t = 0; t < e; ++t) r *= x;
  return r;
}

// exponents (a, b) of monomial q: by total degree, then descending a
__device__ __forceinline__ void mono_exp(int q, int& a, int& b) {
  int d = 0;
  while ((d + 1) * (d + 2) / 2 <= q) ++d;
  b = q - d * (d + 1) / 2;
  a = d - b;
}

template <int SMAX>
__global__ __launch_bounds__(64 * kWaves) void k_phs_weights(int64_t nsys, int ns, int L, int m,
                                                            const double* __restrict__ xyz,
                                                            const double* __restrict__ nrm,
                                                            const int32_t* __restrict__ sten,
                                                            double* __restrict__ w, int* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t sys = int64_t(blockIdx.x) * kWaves + wv;
  const bool active = sys < nsys;  // uniform per wavefront
  const int S = ns + L;
  __shared__ double xs[kWaves][64][2];

  // tangent frame of the centre (Sec. 2.1) and this lane's projected point
  double px = 0.0, py = 0.0;
  if (active) {
    const int32_t* st = sten + sys * ns;
    const int ci = st[0];
    double n0 = nrm[3 * ci], n1 = nrm[3 * ci + 1], n2 = nrm[3 * ci + 2];
    double nn = sqrt(fma(n0, n0, fma(n1, n1, n2 * n2)));
    n0 /= nn;
    n1 /= nn;
    n2 /= nn;
    int ax = 0;
    if (fabs(n1) < fabs(n0)) ax = 1;
    if (fabs(n2) < fabs(ax == 0 ? n0 : n1)) ax = 2;
    double nax = ax == 0 ? n0 : (ax == 1 ? n1 : n2);
    double t1x = (ax == 0 ? 1.0 : 0.0) - nax * n0;
    double t1y = (ax == 1 ? 1.0 : 0.0) - nax * n1;
    double t1z = (ax == 2 ? 1.0 : 0.0) - nax * n2;
    double l1 = sqrt(t1x * t1x + t1y * t1y + t1z * t1z);
    t1x /= l1;
    t1y /= l1;
    t1z /= l1;
    double t2x = n1 * t1z - n2 * t1y, t2y = n2 * t1x - n0 * t1z, t2z = n0 * t1y - n1 * t1x;
    if (lane < ns) {
      const int j = st[lane];
      double dx = xyz[3 * j] - xyz[3 * ci], dy = xyz[3 * j + 1] - xyz[3 * ci + 1], dz = xyz[3 * j + 2] - xyz[3 * ci + 2];
      px = t1x * dx + t1y * dy + t1z * dz;
      py = t2x * dx + t2y * dy + t2z * dz;
    }
  }
  double r = sqrt(px * px + py * py);
  double s = r;
  for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off, 64));
  if (!(s > 0.0)) s = 1.0;
  px /= s;
  py /= s;
  r /= s;
  xs[wv][lane][0] = px;
  xs[wv][lane][1] = py;
  __syncthreads();

  // row `lane` of [M | rhs]; columns S..SMAX-1 are zero padding, rhs in a[SMAX]
  double a[SMAX + 1];
  int qa = 0, qb = 0;
  if (lane >= ns && lane < S) mono_exp(lane - ns, qa, qb);
#pragma unroll
  for (int k = 0; k < SMAX; ++k) {
    double v = 0.0;
    if (k < S) {
      const double xk = xs[wv][k][0], yk = xs[wv][k][1];
      if (lane < ns) {
        if (k < ns) {
          double dx = px - xk, dy = py - yk;
          v = ipow_d(sqrt(dx * dx + dy * dy), m);
        } else {
          int ea, eb;
          mono_exp(k - ns, ea, eb);
          v = ipow_d(px, ea) * ipow_d(py, eb);
        }
      } else if (lane < S && k < ns) {
        v = ipow_d(xk, qa) * ipow_d(yk, qb);
      }
    }
    a[k] = v;
  }
  a[SMAX] = lane < ns ? double(m) * double(m) * ipow_d(r, m - 2)
                      : ((lane < S && ((qa == 2 && qb == 0) || (qa == 0 && qb == 2))) ? 2.0 : 0.0);

  double amax = 0.0;
#pragma unroll
  for (int k = 0; k < SMAX; ++k) amax = fmax(amax, fabs(a[k]));
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  const double tiny = amax * 1e-13;

  bool used = lane >= S;
  int kpos = -1;
  bool singular = false;
#pragma unroll
  for (int k = 0; k < SMAX; ++k) {
    if (k < S) {
      const double v = a[k];
      // pivot: the unused lane with the largest |a_lk|, ties to the lower lane.
      // |a| as a non-negative double orders like its bit pattern: compare the
      // high words (+1 so that used lanes, keyed 0, never win), then the low
      // words among the lanes holding the maximum, then take the lowest lane.
      const uint64_t bits = __builtin_bit_cast(uint64_t, fabs(v));
      const uint32_t khi = used ? 0u : uint32_t(bits >> 32) + 1u;
      const uint32_t mhi = wave_max_u32(khi);
      const bool top = khi == mhi;
      const uint32_t mlo = wave_max_u32(top ? uint32_t(bits) : 0u);
      const int bl = int(__builtin_ctzll(__ballot(top && uint32_t(bits) == mlo)));
      const double bv = used ? -1.0 : fabs(v);
      if (!(readlane_d(bv, bl) > tiny)) singular = true;
      const double piv = readlane_d(v, bl);
      const double mlt = (lane == bl) ? 0.0 : v / piv;
#pragma unroll
      for (int j = k + 1; j <= SMAX; ++j) a[j] = fma(-mlt, readlane_d(a[j], bl), a[j]);
      if (lane == bl) {
        used = true;
        kpos = k;
      }
    }
  }
  // solution component of this row: rhs / diagonal
  double diag = 1.0;
#pragma unroll
  for (int k = 0; k < SMAX; ++k)
    if (k == kpos) diag = a[k];
  if (active) {
    if (singular) {
      if (lane == 0) atomicMax(status, 1);
    } else if (kpos >= 0 && kpos < ns) {
      w[sys * ns + kpos] = (a[SMAX] / diag) / (s * s);
    }
  }
}

#define HIPOK(x)                                                                                   \
  do {                                                                                             \
    hipError_t e_ = (x);                                                                           \
    if (e_ != hipSuccess) throw Error(MGM_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

// Device pointers; launches on `st`. Throws on invalid sizes.
void batched_phs_weights_device(const double* d_xyz, const double* d_nrm, const int32_t* d_sten, int64_t nsys, int ns,
                                int phs_order, int deg, double* d_w, int* d_status, hipStream_t st) {
  const int L = (deg + 1) * (deg + 2) / 2;
  if (ns < 1 || ns + L > 64) throw Error(MGM_E_ARG, "device weights need stencil_size + L <= 64");
  if (deg < 0 || deg > 6 || phs_order < 0 || phs_order > 6) throw Error(MGM_E_ARG, "phs_order/poly_degree out of range");
  if (nsys <= 0) return;
  if ((nsys + kWaves - 1) / kWaves > 0x7fffffff) throw Error(MGM_E_ARG, "too many systems for one launch");
  const int m = 2 * phs_order + 1;
  const unsigned blocks = unsigned((nsys + kWaves - 1) / kWaves);
  // the register row is sized for the system: S = 60 (50 points, degree 3) needs 61 doubles, not 65
  const int S = ns + L;
  if (S <= 32)
    hipLaunchKernelGGL(k_phs_weights<32>, dim3(blocks), dim3(64 * kWaves), 0, st, nsys, ns, L, m, d_xyz, d_nrm, d_sten,
                       d_w, d_status);
  else if (S <= 48)
    hipLaunchKernelGGL(k_phs_weights<48>, dim3(blocks), dim3(64 * kWaves), 0, st, nsys, ns, L, m, d_xyz, d_nrm, d_sten,
                       d_w, d_status);
  else if (S <= 60)
    hipLaunchKernelGGL(k_phs_weights<60>, dim3(blocks), dim3(64 * kWaves), 0, st, nsys, ns, L, m, d_xyz, d_nrm, d_sten,
                       d_w, d_status);
  else
    hipLaunchKernelGGL(k_phs_weights<64>, dim3(blocks), dim3(64 * kWaves), 0, st, nsys, ns, L, m, d_xyz, d_nrm, d_sten,
                       d_w, d_status);
  HIPOK(hipGetLastError());
}

// ------------------------------------------------- allocation-free variant
// Device scratch of mgm_batched_weights_noalloc: int 0 is the flag that the
// weight kernel raises for a singular system (the buffer that
// mgm_batched_weights allocates per call). A file-scope device array: every
// GPU the library runs on holds its own copy until the process ends, and
// host code may only use the per-device address that hipGetSymbolAddress
// returns, never the array's name.
constexpr size_t kNoallocScratchBytes = 256;
static __device__ __align__(256) int scratch[kNoallocScratchBytes / sizeof(int)];

namespace {

constexpr size_t kNoallocStatusBytes = sizeof(int);  // what one call uses, whatever the batch size
static_assert(kNoallocStatusBytes <= kNoallocScratchBytes, "status word must fit the scratch");

__global__ void k_clear_status(int* status) { status[0] = 0; }

std::mutex g_scratch_mu;
std::vector<int*> g_scratch_dev;  // scratch address per device ordinal, looked up once

// The scratch address on the current device (the one whose buffers the call
// receives), looked up on the first call on that device.
int* scratch_on_current_device() {
  int dev = -1;
  HIPOK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev >= int(g_scratch_dev.size())) g_scratch_dev.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPOK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(MGM_E_HIP, "no device address for the weight solver's scratch");
    g_scratch_dev[dev] = static_cast<int*>(p);
  }
  return g_scratch_dev[dev];
}

}  // namespace

}  // namespace mgm

extern "C" mgm_status mgm_batched_weights_noalloc(const double* d_xyz, const double* d_normals, int64_t n_points,
                                                  const int32_t* d_stencils, int64_t n_systems, int32_t stencil_size,
                                                  int32_t phs_order, int32_t poly_degree, double* d_weights,
                                                  void* stream) {
  using namespace mgm;
  if (!d_xyz || !d_normals || !d_stencils || !d_weights || n_points < 1 || n_systems < 0 || stencil_size < 1 ||
      stencil_size > n_points) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  mgm_status res = MGM_OK;
  const mgm_status s = guard([&] {
    hipStream_t st = static_cast<hipStream_t>(stream);
    int* status = scratch_on_current_device();
    // the array keeps the previous call's flag: clear it on the stream first
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, st, status);
    HIPOK(hipGetLastError());
    batched_phs_weights_device(d_xyz, d_normals, d_stencils, n_systems, stencil_size, phs_order, poly_degree,
                               d_weights, status, st);
    int h_status = 0;
    HIPOK(hipMemcpyAsync(&h_status, status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPOK(hipStreamSynchronize(st));
    if (h_status) {
      g_last_error = "a stencil system is singular";
      res = MGM_E_STENCIL_SINGULAR;
    }
  });
  return s != MGM_OK ? s : res;
}
