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

// x^e with the exponent fixed at compile time when EC > 0 (the same products
// in the same order as ipow_d, so the same bits), else e
template <int EC>
__device__ __forceinline__ double ipow_c(double x, int e) {
  if constexpr (EC > 0) {
    double r = 1.0;
#pragma unroll
    for (int t = 0; t < EC; ++t) r *= x;
    return r;
  } else {
    return ipow_d(x, e);
  }
}

// Square root of a scaled squared distance x: zero, or at least 2^-767 (the
// points lie in the unit disc, and two distinct FP64 points there are at
// least ~1e-16 apart), so no range scaling is needed. Goldschmidt's iteration
// from the hardware reciprocal square root y ~ 1/sqrt(x): g = x y and
// h = y / 2 converge to sqrt(x) and 1/(2 sqrt(x)); one coupled step, then two
// corrections g += (x - g^2) h. These are the steps of the correctly rounded
// sqrt() of this target without its scaling of inputs below 2^-767, so in
// this range the bits are sqrt()'s. x = 0 gives 0 (the iteration would give
// NaN).
__device__ __forceinline__ double sqrt_dist(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = y * 0.5;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  g = fma(d, h, g);
  return x == 0.0 ? 0.0 : g;
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

// ------------------------------------------------------ MFMA blocked variant
// The same Gauss-Jordan elimination with partial pivoting, blocked by panels
// of 4 columns so that the update of the remaining columns is a 64 x 4 by
// 4 x 64 product on the FP64 matrix cores (v_mfma_f64_16x16x4f64). One
// wavefront per system; the 64 x 64 matrix (the system padded with identity
// rows and columns) stays in the MFMA accumulator layout for the whole solve:
// tile (bi, bj) = rows 16bi.., columns 16bj..; lane 16g + c holds, in its
// register v of that tile, row 16bi + 4v + g, column 16bj + c. The right-hand
// side stays in rows (lane r holds row r).
// Per panel p (columns 4p .. 4p+3):
//  1. its 64 x 4 columns go through LDS into rows (lane r: row r);
//  2. four pivot steps on them (unused row with the largest |entry|, ties to
//     the lower row): multipliers M[r][k], pivot rows b_k;
//  3. the pivot rows' current entries B (4 x 64, through LDS) become
//     U = Lambda^-1 B, Lambda the unit lower triangle of the multipliers the
//     panel applied to its own pivot rows (U[k] is pivot row b_k as it stood
//     at step k); columns of this and earlier panels are set to zero in U;
//  4. every row r: A[r][:] -= sum_k M[r][k] U[k][:], as MFMA tiles.
// This is the unblocked elimination's arithmetic reassociated per panel.
// After the last panel each pivot row holds one nonzero and x = rhs / pivot.
// The 64 x 64 FP64 matrix takes 128 registers of every lane; the register
// bound of three wavefronts per SIMD (168) spills a few values of the
// assembly phase, which costs less than the latency two wavefronts leave
// exposed (measured: 12.2 against 15.5 ms for 500,000 systems of 60).
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kMWaves = 4;    // systems (wavefronts) per block
constexpr int kMonoMax = 16;  // monomials per point in the table: degree <= 4

// Order the LDS accesses of the lanes of one wavefront (no hardware wait).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The mixed-precision kernel's set-up, the same arithmetic as the FP64
// matrix-core kernel's (which keeps its own inline copy: factored out, it
// spilled more registers and took 4% longer). The centre's tangent frame
// (Sec. 2.1) and this lane's projected stencil point, scaled by the stencil
// radius s (returned with the lane's scaled distance r), to xsw[lane]. Inactive wavefronts compute on zeros. Its
// monomials (total degree, then descending power of x) then go to
// mono[lane * kMonoMax ..] (phs_monomials), so that the polynomial entries
// are table reads.
__device__ __forceinline__ void phs_stencil_points(bool active, int64_t sys, int ns, int lane,
                                                   const double* __restrict__ xyz, const double* __restrict__ nrm,
                                                   const int32_t* __restrict__ sten, double (*xsw)[2], double& r_out,
                                                   double& s_out) {
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
  xsw[lane][0] = px;
  xsw[lane][1] = py;
  r_out = r;
  s_out = s;
}

// the monomials of this lane's scaled point (after phs_stencil_points)
__device__ __forceinline__ void phs_monomials(int deg, int lane, const double (*xsw)[2], double* mono) {
  const double px = xsw[lane][0], py = xsw[lane][1];
  int q = 0;  // (deg + 1)(deg + 2) / 2 = L <= kMonoMax monomials (checked on the host)
  for (int d = 0; d <= deg; ++d)
    for (int b = 0; b <= d; ++b, ++q) mono[lane * kMonoMax + q] = ipow_d(px, d - b) * ipow_d(py, b);
}

// Entry (row, col) of the system padded to 64 x 64 with identity rows and
// columns, column point (xc, yc): the PHS block, P (row a point, col a
// monomial) or P^T, the zero block; `inside` is false on the padding. Every
// candidate is computed and the result selected, without branches.
template <int MC>
__device__ __forceinline__ double phs_entry(const double (*xsw)[2], const double* mono, int row, int col, double xc,
                                            double yc, int ns, int S, int m, bool& inside) {
  const double dx = xsw[row][0] - xc, dy = xsw[row][1] - yc;
  const double phs = ipow_c<MC>(sqrt_dist(dx * dx + dy * dy), m);
  const bool rp = row < ns;
  const int pt = rp ? row : col, mq = (rp ? col : row) - ns;
  const double pq = mono[pt * kMonoMax + min(max(mq, 0), kMonoMax - 1)];
  inside = row < S && col < S;
  const double vin = (row < ns && col < ns) ? phs : ((row < ns) != (col < ns) ? pq : 0.0);
  return inside ? vin : (row == col ? 1.0 : 0.0);
}

// right-hand side (eq. rbf_fd_lap) of row `lane`: Lap r^m at the points, Lap p(0)
// for the monomials, zero on the padding
template <int MC>
__device__ __forceinline__ double phs_rhs(int lane, double r, int ns, int S, int m) {
  if (lane < ns) return double(m) * double(m) * ipow_c<(MC > 2 ? MC - 2 : 0)>(r, m - 2);
  if (lane < S) {
    int qa, qb;
    mono_exp(lane - ns, qa, qb);
    return ((qa == 2 && qb == 0) || (qa == 0 && qb == 2)) ? 2.0 : 0.0;
  }
  return 0.0;
}

// PHS exponent m fixed at compile time (MC > 0) or read from m; likewise the
// stencil size (NSC > 0) and the polynomial degree (DEGC >= 0)
template <int MC, int NSC = 0, int DEGC = -1>
__global__ __launch_bounds__(64 * kMWaves, 3) void k_phs_weights_mfma(int64_t nsys, int ns_rt, int deg_rt, int L_rt,
                                                                 int m, const double* __restrict__ xyz,
                                                                 const double* __restrict__ nrm,
                                                                 const int32_t* __restrict__ sten,
                                                                 double* __restrict__ w, int* __restrict__ status) {
  const int ns = NSC > 0 ? NSC : ns_rt;
  const int deg = DEGC >= 0 ? DEGC : deg_rt;
  const int L = DEGC >= 0 ? (DEGC + 1) * (DEGC + 2) / 2 : L_rt;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t sys = int64_t(blockIdx.x) * kMWaves + wv;
  const bool active = sys < nsys;  // uniform per wavefront
  const int S = ns + L;
  __shared__ double xs[kMWaves][64][2];
  // per wavefront: the monomial table, then per panel the panel rows / the A
  // operand (-M, 64 x 4) and the pivot rows B / U (4 x 64)
  __shared__ double scr[kMWaves][64 * kMonoMax];

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
  wave_sync();

  // the monomials of this lane's point (total degree, then descending power
  // of x), so that the polynomial entries are table reads
  double* mono = scr[wv];  // kMonoMax per point
  {
    int q = 0;  // (deg + 1)(deg + 2) / 2 = L <= kMonoMax monomials (checked on the host)
    for (int d = 0; d <= deg; ++d)
      for (int b = 0; b <= d; ++b, ++q) mono[lane * kMonoMax + q] = ipow_d(px, d - b) * ipow_d(py, b);
  }
  wave_sync();
  // the padded system in the accumulator layout
  dbl4 acc[4][4];
  double amax = 0.0;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    const int col = 16 * bj + c;
    const double xc = xs[wv][col][0], yc = xs[wv][col][1];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * bi + 4 * v + g;
        const double dx = xs[wv][row][0] - xc, dy = xs[wv][row][1] - yc;
        const double phs = ipow_c<MC>(sqrt_dist(dx * dx + dy * dy), m);
        // P (row a point, col a monomial) or P^T (row a monomial, col a point)
        const bool rp = row < ns;
        const int pt = rp ? row : col, mq = (rp ? col : row) - ns;
        const double pq = mono[pt * kMonoMax + min(max(mq, 0), kMonoMax - 1)];
        double val;
        if (row < S && col < S) {
          val = (row < ns && col < ns) ? phs : ((row < ns) != (col < ns) ? pq : 0.0);
          amax = fmax(amax, fabs(val));
        } else {
          val = row == col ? 1.0 : 0.0;  // padding: identity
        }
        acc[bi][bj][v] = val;
      }
    }
  }
  wave_sync();  // the monomial table's space is reused below
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  const double tiny = amax * 1e-13;
  // right-hand side (eq. rbf_fd_lap), row `lane`
  double rhs = 0.0;
  if (lane < ns) {
    rhs = double(m) * double(m) * ipow_c<(MC > 2 ? MC - 2 : 0)>(r, m - 2);
  } else if (lane < S) {
    int qa, qb;
    mono_exp(lane - ns, qa, qb);
    rhs = ((qa == 2 && qb == 0) || (qa == 0 && qb == 2)) ? 2.0 : 0.0;
  }

  bool used = false;
  int kpos = -1;
  double diag = 1.0;
  bool singular = false;
  double(*pan)[4] = reinterpret_cast<double(*)[4]>(scr[wv]);          // 64 x 4
  double(*ub)[64] = reinterpret_cast<double(*)[64]>(scr[wv] + 64 * 4);  // 4 x 64
  const int np = (S + 3) / 4;
  for (int p = 0; p < np; ++p) {
    const int bjp = p >> 2, co = (p & 3) * 4;
    // 1. the panel's columns into rows
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
      if (bj == bjp && c >= co && c < co + 4) {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int v = 0; v < 4; ++v) pan[16 * bi + 4 * v + g][c - co] = acc[bi][bj][v];
      }
    wave_sync();
    double pr[4], mk[4];
    int bk[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) pr[j] = pan[lane][j];
    // 2. pivot steps on the panel
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double v = pr[k];
      // pivot: the unused row whose |v|, rounded to FP32, is largest (a
      // non-negative float orders like its bit pattern; +1 so that used
      // rows, keyed 0, never win), ties to the lowest row: one wave-wide
      // maximum instead of an exact FP64 comparison in two passes
      const uint32_t key = used ? 0u : __builtin_bit_cast(uint32_t, float(fabs(v))) + 1u;
      const uint32_t kmax = wave_max_u32(key);
      const int bl = int(__builtin_ctzll(__ballot(key == kmax)));
      const double piv = readlane_d(v, bl);
      if (4 * p + k < S && !(fabs(piv) > tiny)) singular = true;
      const double rpiv = 1.0 / piv;
      const double mlt = lane == bl ? 0.0 : v * rpiv;
#pragma unroll
      for (int j = k + 1; j < 4; ++j) pr[j] = fma(-mlt, readlane_d(pr[j], bl), pr[j]);
      mk[k] = mlt;
      bk[k] = bl;
      if (lane == bl) {
        used = true;
        kpos = 4 * p + k;
        diag = piv;
      }
    }
    // 3. pivot rows B (current entries) into LDS, then U = Lambda^-1 B. The
    // pivot row's register (bi, v) is uniform: one switch (a short tree of
    // scalar branches) instead of a test per register
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rb = bk[k];
      if (g == (rb & 3)) {
#define PIVOT_ROW(BI, V)                                                          \
  case 4 * BI + V:                                                                \
    _Pragma("unroll") for (int bj = 0; bj < 4; ++bj) ub[k][16 * bj + c] = acc[BI][bj][V]; \
    break;
        switch (rb >> 2) {
          PIVOT_ROW(0, 0) PIVOT_ROW(0, 1) PIVOT_ROW(0, 2) PIVOT_ROW(0, 3)
          PIVOT_ROW(1, 0) PIVOT_ROW(1, 1) PIVOT_ROW(1, 2) PIVOT_ROW(1, 3)
          PIVOT_ROW(2, 0) PIVOT_ROW(2, 1) PIVOT_ROW(2, 2) PIVOT_ROW(2, 3)
          PIVOT_ROW(3, 0) PIVOT_ROW(3, 1) PIVOT_ROW(3, 2) PIVOT_ROW(3, 3)
          default: break;
        }
#undef PIVOT_ROW
      }
    }
    double lam[4][4];  // lam[k][q] = multiplier of pivot row b_k at step q < k
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < k; ++q) lam[k][q] = readlane_d(mk[q], bk[k]);
    wave_sync();
    double u[4], urhs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      u[k] = ub[k][lane];
      urhs[k] = readlane_d(rhs, bk[k]);
#pragma unroll
      for (int q = 0; q < k; ++q) {
        u[k] = fma(-lam[k][q], u[q], u[k]);
        urhs[k] = fma(-lam[k][q], urhs[q], urhs[k]);
      }
    }
    const bool done_col = lane < 4 * p + 4;  // this lane's column is eliminated already
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      ub[k][lane] = done_col ? 0.0 : u[k];
      rhs = fma(-mk[k], urhs[k], rhs);
      pan[lane][k] = -mk[k];
    }
    wave_sync();
    // 4. the update on the matrix cores: A operand lane 16k + i = -M[16bi + i][k],
    //    B operand lane 16k + j = U[k][16bj + j]
    double aop[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) aop[bi] = pan[16 * bi + c][g];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
      if (bj >= bjp) {
        const double bop = ub[g][16 * bj + c];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[bi], bop, acc[bi][bj], 0, 0, 0);
      }
    wave_sync();  // the next panel reuses pan and ub
  }
  if (active) {
    if (singular) {
      if (lane == 0) atomicMax(status, 1);
    } else if (kpos >= 0 && kpos < ns) {
      w[sys * ns + kpos] = (rhs / diag) / (s * s);
    }
  }
}

// --------------------------------- FP32 matrix cores with FP64 refinement
// The same system, eliminated in FP32 on the matrix cores and refined in FP64
// (mixed-precision iterative refinement). Gauss-Jordan with partial pivoting,
// in panels of 4 columns as above, runs on [A | I] (64 x 128 in FP32, tiles
// bj = 0..3 holding A and 4..7 the identity, v_mfma_f32_16x16x4f32 updates;
// the FP32 accumulator layout is lane 16g + c, register v -> row 4g + v,
// column c of a tile). Afterwards pivot row r (the row chosen for column k_r)
// holds d_r e_{k_r}^T in its A part and T_r in its I part, with T A = D P
// (P the permutation): A^-1 = (rows T_r / d_r, placed at k_r). Then, from
// x = 0: res = b - A x in FP64 (row r assembled again on lane r) and
// x_{k_r} += (T_r . res) / d_r, until a correction is below 2^-50 of the
// largest |x| or no longer halves the one before (the FP64 residual's
// rounding is reached), at most kMaxSweeps solves. Each correction contracts
// the error by about cond(A) eps_fp32: ~2e-3 a sweep for r^3 stencils
// (condition numbers ~3e4). A system whose last correction still exceeds
// 1e-8 of |x| (the FP32 elimination too inaccurate for the refinement to
// converge) is reported like a singular one.
typedef float flt4 __attribute__((ext_vector_type(4)));
constexpr int kMaxSweeps = 10;

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// compile-time PHS exponent, stencil size and degree as in k_phs_weights_mfma
template <int MC, int NSC = 0, int DEGC = -1>
__global__ __launch_bounds__(64 * kMWaves, 3) void k_phs_weights_mixed(int64_t nsys, int ns_rt, int deg_rt, int L_rt,
                                                                  int m, const double* __restrict__ xyz,
                                                                  const double* __restrict__ nrm,
                                                                  const int32_t* __restrict__ sten,
                                                                  double* __restrict__ w, int* __restrict__ status) {
  const int ns = NSC > 0 ? NSC : ns_rt;
  const int deg = DEGC >= 0 ? DEGC : deg_rt;
  const int L = DEGC >= 0 ? (DEGC + 1) * (DEGC + 2) / 2 : L_rt;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t sys = int64_t(blockIdx.x) * kMWaves + wv;
  const bool active = sys < nsys;  // uniform per wavefront
  const int S = ns + L;
  __shared__ double xs[kMWaves][64][2];
  __shared__ double mono_s[kMWaves][64 * kMonoMax];  // kept for the residuals
  // per wavefront: the panel (-M, 64 x 4) and the pivot rows (4 x 128), FP32;
  // after the elimination the residual, the solution and the correction
  __shared__ double work[kMWaves][(64 * 4 + 4 * 128) / 2];

  double r, s;
  phs_stencil_points(active, sys, ns, lane, xyz, nrm, sten, xs[wv], r, s);
  wave_sync();
  const double* mono = mono_s[wv];
  phs_monomials(deg, lane, xs[wv], mono_s[wv]);
  wave_sync();
  flt4 acc[4][8];
  double amax = 0.0;
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    const int col = 16 * bj + c;
    const double xc = xs[wv][col][0], yc = xs[wv][col][1];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        bool inside;
        const double val = phs_entry<MC>(xs[wv], mono, 16 * bi + 4 * g + v, col, xc, yc, ns, S, m, inside);
        if (inside) amax = fmax(amax, fabs(val));
        acc[bi][bj][v] = float(val);
      }
    }
  }
#pragma unroll
  for (int bj = 4; bj < 8; ++bj)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[bi][bj][v] = (16 * bi + 4 * g + v == 16 * (bj - 4) + c) ? 1.0f : 0.0f;
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  const double tiny = amax * 1e-13;
  const double b = phs_rhs<MC>(lane, r, ns, S, m);

  bool used = false;
  int kpos = -1;
  float diag = 1.0f;
  bool singular = false;
  float(*pan)[4] = reinterpret_cast<float(*)[4]>(work[wv]);                // 64 x 4
  float(*ub)[128] = reinterpret_cast<float(*)[128]>(work[wv] + 64 * 4 / 2);  // 4 x 128
  const int np = (S + 3) / 4;
  for (int p = 0; p < np; ++p) {
    const int bjp = p >> 2, co = (p & 3) * 4;
    // 1. the panel's columns into rows
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
      if (bj == bjp && c >= co && c < co + 4) {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int v = 0; v < 4; ++v) pan[16 * bi + 4 * g + v][c - co] = acc[bi][bj][v];
      }
    wave_sync();
    float pr[4], mk[4];
    int bk[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) pr[j] = pan[lane][j];
    // 2. pivot steps on the panel (the unused row with the largest |entry|,
    //    ties to the lowest row)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float v = pr[k];
      const uint32_t key = used ? 0u : __builtin_bit_cast(uint32_t, fabsf(v)) + 1u;
      const uint32_t kmax = wave_max_u32(key);
      const int bl = int(__builtin_ctzll(__ballot(key == kmax)));
      const float piv = readlane_f(v, bl);
      if (4 * p + k < S && !(fabs(double(piv)) > tiny)) singular = true;
      const float rpiv = 1.0f / piv;
      const float mlt = lane == bl ? 0.0f : v * rpiv;
#pragma unroll
      for (int j = k + 1; j < 4; ++j) pr[j] = fmaf(-mlt, readlane_f(pr[j], bl), pr[j]);
      mk[k] = mlt;
      bk[k] = bl;
      if (lane == bl) {
        used = true;
        kpos = 4 * p + k;
        diag = piv;
      }
    }
    // 3. the pivot rows' current entries (A and I parts), then U = Lambda^-1 B
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rb = bk[k];
      if (g == ((rb >> 2) & 3)) {
        // the pivot row's register (bi, v) is uniform: one switch
#define PIVOT_ROW32(BI, V)                                                        \
  case 4 * BI + V:                                                                \
    _Pragma("unroll") for (int bj = 0; bj < 8; ++bj) ub[k][16 * bj + c] = acc[BI][bj][V]; \
    break;
        switch (((rb >> 4) << 2) | (rb & 3)) {
          PIVOT_ROW32(0, 0) PIVOT_ROW32(0, 1) PIVOT_ROW32(0, 2) PIVOT_ROW32(0, 3)
          PIVOT_ROW32(1, 0) PIVOT_ROW32(1, 1) PIVOT_ROW32(1, 2) PIVOT_ROW32(1, 3)
          PIVOT_ROW32(2, 0) PIVOT_ROW32(2, 1) PIVOT_ROW32(2, 2) PIVOT_ROW32(2, 3)
          PIVOT_ROW32(3, 0) PIVOT_ROW32(3, 1) PIVOT_ROW32(3, 2) PIVOT_ROW32(3, 3)
          default: break;
        }
#undef PIVOT_ROW32
      }
    }
    float lam[4][4];  // lam[k][q] = multiplier of pivot row b_k at step q < k
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < k; ++q) lam[k][q] = readlane_f(mk[q], bk[k]);
    wave_sync();
    float u[4][2];  // columns lane (A part) and 64 + lane (I part)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      u[k][0] = ub[k][lane];
      u[k][1] = ub[k][64 + lane];
#pragma unroll
      for (int q = 0; q < k; ++q) {
        u[k][0] = fmaf(-lam[k][q], u[q][0], u[k][0]);
        u[k][1] = fmaf(-lam[k][q], u[q][1], u[k][1]);
      }
    }
    const bool done_col = lane < 4 * p + 4;  // this lane's A column is eliminated already
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      ub[k][lane] = done_col ? 0.0f : u[k][0];
      ub[k][64 + lane] = u[k][1];
      pan[lane][k] = -mk[k];
    }
    wave_sync();
    // 4. the update on the matrix cores (A part from the panel's tile on, all of the I part)
    float aop[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) aop[bi] = pan[16 * bi + c][g];
#pragma unroll
    for (int bj = 0; bj < 8; ++bj)
      if (bj >= bjp) {
        const float bop = ub[g][16 * bj + c];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[bi], bop, acc[bi][bj], 0, 0, 0);
      }
    wave_sync();  // the next panel reuses pan and ub
  }
  // 5. solve and refine in FP64
  double* rs = work[wv];        // residual, by row
  double* xsol = work[wv] + 64;  // solution, by column
  double* dv = work[wv] + 128;   // correction, by row
  xsol[lane] = 0.0;
  double res = b;
  bool converged = false;
  double dprev = 0.0, xlast = 0.0;
  for (int it = 0; it < kMaxSweeps && !converged; ++it) {
    if (it > 0) {
      double ax = 0.0;  // row `lane` of A times x, the entries assembled again
      for (int j = 0; j < S; ++j) {
        bool inside;
        const double a = phs_entry<MC>(xs[wv], mono, lane, j, xs[wv][j][0], xs[wv][j][1], ns, S, m, inside);
        ax = fma(a, xsol[j], ax);
      }
      res = lane < S ? b - ax : 0.0;
    }
    rs[lane] = res;
    wave_sync();
    double rc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) rc[t] = rs[16 * t + c];
    double pd[4][4];  // T row . res over this lane's four columns, rows 16 bi + 4g + v
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t0 = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) t0 = fma(double(acc[bi][4 + t][v]), rc[t], t0);
        pd[bi][v] = t0;
      }
    // sum over the 16 lanes of each row group (the columns), in a fixed tree
#pragma unroll
    for (int off = 1; off < 16; off <<= 1)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) pd[bi][v] += __shfl_xor(pd[bi][v], off, 64);
    if (c == 0) {
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) dv[16 * bi + 4 * g + v] = pd[bi][v];
    }
    wave_sync();
    double dmax = 0.0, xmax = 0.0;
    if (kpos >= 0) {
      const double dx = dv[lane] / double(diag);
      const double xn = xsol[kpos] + dx;
      xsol[kpos] = xn;
      if (kpos < S) {
        dmax = fabs(dx);
        xmax = fabs(xn);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
      xmax = fmax(xmax, __shfl_xor(xmax, off, 64));
    }
    // the same on every lane
    converged = it > 0 && (dmax <= 0x1.0p-50 * xmax || dmax > 0.5 * dprev);
    dprev = dmax;
    xlast = xmax;
    wave_sync();
  }
  if (!(dprev <= 1e-8 * xlast)) singular = true;
  if (active) {
    if (singular) {
      if (lane == 0) atomicMax(status, 1);
    } else if (lane < ns) {
      w[sys * ns + lane] = xsol[lane] / (s * s);
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
                                int phs_order, int deg, double* d_w, int* d_status, hipStream_t st, bool mixed) {
  const int L = (deg + 1) * (deg + 2) / 2;
  if (ns < 1 || ns + L > 64) throw Error(MGM_E_ARG, "device weights need stencil_size + L <= 64");
  if (deg < 0 || deg > 6 || phs_order < 1 || phs_order > 6)
    throw Error(MGM_E_ARG, "phs_order must be 1..6 and poly_degree 0..6");
  if (mixed && L > kMonoMax) throw Error(MGM_E_ARG, "the mixed-precision weights need poly_degree <= 4");
  if (nsys <= 0) return;
  if (mixed) {
    if ((nsys + kMWaves - 1) / kMWaves > 0x7fffffff) throw Error(MGM_E_ARG, "too many systems for one launch");
    const dim3 grid(unsigned((nsys + kMWaves - 1) / kMWaves)), block(64 * kMWaves);
    const int mm = 2 * phs_order + 1;
    const bool n50d3 = ns == 50 && deg == 3;
#define PHS_MIXED_K(...)                                                                                          \
  hipLaunchKernelGGL((k_phs_weights_mixed<__VA_ARGS__>), grid, block, 0, st, nsys, ns, deg, L, mm, d_xyz, d_nrm, \
                     d_sten, d_w, d_status)
#define PHS_MIXED(MC) \
  if (n50d3) PHS_MIXED_K(MC, 50, 3); else PHS_MIXED_K(MC);
    switch (mm) {
      case 3: PHS_MIXED(3) break;
      case 5: PHS_MIXED(5) break;
      case 7: PHS_MIXED(7) break;
      default: PHS_MIXED_K(0); break;
    }
#undef PHS_MIXED
#undef PHS_MIXED_K
    HIPOK(hipGetLastError());
    return;
  }
  if ((nsys + kWaves - 1) / kWaves > 0x7fffffff) throw Error(MGM_E_ARG, "too many systems for one launch");
  const int m = 2 * phs_order + 1;
  const unsigned blocks = unsigned((nsys + kWaves - 1) / kWaves);
  // the register row is sized for the system: S = 60 (50 points, degree 3) needs 61 doubles, not 65
  const int S = ns + L;
  if (S > 32 && L <= kMonoMax) {
    // larger systems: blocked elimination with the update on the matrix cores
    const unsigned mblocks = unsigned((nsys + kMWaves - 1) / kMWaves);
    // the common 50-point, degree-3 stencils also with their sizes fixed
    const bool n50d3 = ns == 50 && deg == 3;
#define PHS_MFMA_K(...)                                                                                         \
  hipLaunchKernelGGL((k_phs_weights_mfma<__VA_ARGS__>), dim3(mblocks), dim3(64 * kMWaves), 0, st, nsys, ns, deg, L, m, \
                     d_xyz, d_nrm, d_sten, d_w, d_status)
#define PHS_MFMA(MC) \
  if (n50d3) PHS_MFMA_K(MC, 50, 3); else PHS_MFMA_K(MC);
    switch (m) {
      case 3: PHS_MFMA(3) break;
      case 5: PHS_MFMA(5) break;
      case 7: PHS_MFMA(7) break;
      default: PHS_MFMA_K(0); break;
    }
#undef PHS_MFMA
#undef PHS_MFMA_K
  } else if (S <= 32)
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
  // an empty batch may pass null stencils and weights (it still checks the sizes)
  if (!d_xyz || !d_normals || (n_systems > 0 && (!d_stencils || !d_weights)) || n_points < 1 || n_systems < 0 ||
      stencil_size < 1 || stencil_size > n_points) {
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
                               d_weights, status, st, false);
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
