// Preprocessing steps on the device (Alg. 2): exact k-nearest-neighbour
// searches (stencils, Sec. 2; interpolation neighbours, Sec. 3), the sparse
// products of the Galerkin operator R L P (eq. galerkin) and the DSATUR
// colouring of the smoother's patch graphs. All give the host path's results
// bit for bit: the searches return the unique k smallest keys
// (d2, index) with d2 = ((dx*dx) + (dy*dy)) + dz*dz rounded the same way, and
// every product entry is summed from 0.0 in the host's order (row of the left
// factor ascending, then row of the right factor ascending), one rounding per
// multiply and per add. This file is compiled without floating-point
// contraction (no fused multiply-add), like the host sources.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <limits>

#include "ctx.h"

namespace mgm {
namespace {

struct GridDev {
  double lo[3];
  double h;
  int dim[3];
};

__device__ __forceinline__ int grid_coord(const GridDev& g, double x, int a) {
  const double t = floor((x - g.lo[a]) / g.h);
  if (!(t >= 0)) return 0;
  if (t >= g.dim[a] - 1) return g.dim[a] - 1;
  return int(t);
}

__device__ __forceinline__ bool key_less(double a, int32_t ia, double b, int32_t ib) {
  return a < b || (a == b && ia < ib);
}

// One thread per query (queries visited in cell order through qord, so the
// lanes of a wave scan neighbouring cells). The current k best keys are kept
// sorted in LDS, slot s of lane t at s * TPB + t. Cells are scanned in rings
// of growing Chebyshev radius R; the search stops once the k-th key lies
// strictly inside the ball that the scanned cube contains (with a relative
// margin far above the rounding of d2), or the cube covers the grid.
template <int KMAX, int TPB>
__global__ __launch_bounds__(TPB) void k_knn(int64_t nq, int k, const int32_t* __restrict__ qord,
                                             const double* __restrict__ qxyz, const double* __restrict__ sxyz,
                                             const int32_t* __restrict__ pts, const int32_t* __restrict__ start,
                                             GridDev g, int32_t* __restrict__ idx, double* __restrict__ d2o) {
  __shared__ double kd[KMAX * TPB];
  __shared__ int32_t ki[KMAX * TPB];
  const int lane = threadIdx.x;
  const int64_t t = int64_t(blockIdx.x) * TPB + lane;
  if (t >= nq) return;  // no barrier below
  const int64_t q = qord[t];
  const double qx = qxyz[3 * q], qy = qxyz[3 * q + 1], qz = qxyz[3 * q + 2];
  const double qa[3] = {qx, qy, qz};
  const int c[3] = {grid_coord(g, qx, 0), grid_coord(g, qy, 1), grid_coord(g, qz, 2)};
  int cnt = 0;
  for (int R = 0;; ++R) {
    bool covers_all = true;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      if (c[a] - R > 0 || c[a] + R < g.dim[a] - 1) covers_all = false;
      lo[a] = max(0, c[a] - R);
      hi[a] = min(g.dim[a] - 1, c[a] + R);
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          const int ring = max(abs(x - c[0]), max(abs(y - c[1]), abs(z - c[2])));
          if (ring != R) continue;
          const int64_t ci = (int64_t(z) * g.dim[1] + y) * g.dim[0] + x;
          const int32_t s1 = start[ci + 1];
          for (int32_t s = start[ci]; s < s1; ++s) {
            const double dx = sxyz[3 * int64_t(s)] - qx;
            const double dy = sxyz[3 * int64_t(s) + 1] - qy;
            const double dz = sxyz[3 * int64_t(s) + 2] - qz;
            const double dd = (dx * dx + dy * dy) + dz * dz;
            const int32_t j = pts[s];
            int p;
            if (cnt < k) {
              p = cnt++;
            } else if (key_less(dd, j, kd[(k - 1) * TPB + lane], ki[(k - 1) * TPB + lane])) {
              p = k - 1;
            } else {
              continue;
            }
            while (p > 0 && key_less(dd, j, kd[(p - 1) * TPB + lane], ki[(p - 1) * TPB + lane])) {
              kd[p * TPB + lane] = kd[(p - 1) * TPB + lane];
              ki[p * TPB + lane] = ki[(p - 1) * TPB + lane];
              --p;
            }
            kd[p * TPB + lane] = dd;
            ki[p * TPB + lane] = j;
          }
        }
    if (cnt >= k) {
      if (covers_all) break;
      const double kth = kd[(k - 1) * TPB + lane];
      double rcov = INFINITY;
      for (int a = 0; a < 3; ++a) {
        if (c[a] - R > 0) rcov = fmin(rcov, qa[a] - (g.lo[a] + double(c[a] - R) * g.h));
        if (c[a] + R < g.dim[a] - 1) rcov = fmin(rcov, (g.lo[a] + double(c[a] + R + 1) * g.h) - qa[a]);
      }
      if (rcov == INFINITY || kth < rcov * rcov * (1.0 - 1e-12)) break;
    } else if (covers_all) {
      break;
    }
  }
  for (int s = 0; s < k; ++s) {
    idx[q * k + s] = ki[s * TPB + lane];
    d2o[q * k + s] = kd[s * TPB + lane];
  }
}

// Products of row i of A * B in the host's order, keyed (i, column).
__global__ void k_spgemm_count(int32_t n, const int32_t* __restrict__ aptr, const int32_t* __restrict__ acol,
                               const int32_t* __restrict__ bptr, int64_t* __restrict__ cnt) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t s = 0;
  for (int32_t ka = aptr[i]; ka < aptr[i + 1]; ++ka) s += bptr[acol[ka] + 1] - bptr[acol[ka]];
  cnt[i] = s;
}

__global__ void k_spgemm_expand(int32_t n, const int32_t* __restrict__ aptr, const int32_t* __restrict__ acol,
                                const double* __restrict__ aval, const int32_t* __restrict__ bptr,
                                const int32_t* __restrict__ bcol, const double* __restrict__ bval,
                                const int64_t* __restrict__ off, uint64_t* __restrict__ key, double* __restrict__ val) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t o = off[i];
  for (int32_t ka = aptr[i]; ka < aptr[i + 1]; ++ka) {
    const int32_t r = acol[ka];
    const double a = aval[ka];
    for (int32_t kb = bptr[r]; kb < bptr[r + 1]; ++kb) {
      key[o] = (uint64_t(uint32_t(i)) << 32) | uint32_t(bcol[kb]);
      val[o] = a * bval[kb];
      ++o;
    }
  }
}

__global__ void k_run_flags(int64_t m, const uint64_t* __restrict__ key, int32_t* __restrict__ flag) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= m) return;
  flag[t] = (t == 0 || key[t] != key[t - 1]) ? 1 : 0;
}

// One thread per run of equal keys (run r starts at heads[r]): the entry is
// the run's products summed from 0.0 in their order.
__global__ void k_run_sums(int64_t m, int64_t nruns, const int64_t* __restrict__ heads,
                           const uint64_t* __restrict__ key, const double* __restrict__ val,
                           int32_t* __restrict__ row, int32_t* __restrict__ col, double* __restrict__ out) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nruns) return;
  const int64_t b = heads[r];
  const int64_t e = r + 1 < nruns ? heads[r + 1] : m;
  double acc = 0.0;
  for (int64_t t = b; t < e; ++t) acc += val[t];
  row[r] = int32_t(key[b] >> 32);
  col[r] = int32_t(uint32_t(key[b]));
  out[r] = acc;
}

// heads[r] = position of the first element of run r (incl = inclusive count
// of run starts).
__global__ void k_heads(int64_t m, const int32_t* __restrict__ flag, const int32_t* __restrict__ incl,
                        int64_t* __restrict__ heads) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= m) return;
  if (flag[t]) heads[incl[t] - 1] = t;
}

// DSATUR of one patch graph per 64-lane workgroup (Brelaz 1979; the host's
// dsatur_range): each step colours the uncoloured row with the largest
// (saturation, degree, -index), found as a wave maximum of the packed key
// saturation << 20 | degree << 10 | (1023 - local index), with the smallest
// colour absent from its neighbours (a 256-bit mask per row in LDS), then
// marks that colour in its uncoloured neighbours. Patches hold at most
// kDsaturRows rows, so no row needs more than 256 colours.
constexpr int kDsaturRows = 256;
__global__ __launch_bounds__(64) void k_dsatur(const int32_t* __restrict__ pstart, const int32_t* __restrict__ lptr,
                                               const int32_t* __restrict__ ladj, int32_t* __restrict__ lc,
                                               int32_t* __restrict__ pnlc) {
  __shared__ int16_t col[kDsaturRows], sat[kDsaturRows], deg[kDsaturRows];
  __shared__ uint64_t mask[kDsaturRows][4];
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const int v0 = pstart[p];
  const int n = pstart[p + 1] - v0;  // <= kDsaturRows (checked on the host)
  for (int v = lane; v < n; v += 64) {
    col[v] = -1;
    sat[v] = 0;
    deg[v] = int16_t(lptr[v0 + v + 1] - lptr[v0 + v]);
    for (int w = 0; w < 4; ++w) mask[v][w] = 0;
  }
  __syncthreads();
  int maxc = 0;
  for (int step = 0; step < n; ++step) {
    uint32_t best = 0;
    for (int v = lane; v < n; v += 64)
      if (col[v] < 0) best = max(best, (uint32_t(sat[v]) << 20) | (uint32_t(deg[v]) << 10) | uint32_t(1023 - v));
    for (int o = 32; o > 0; o >>= 1) best = max(best, uint32_t(__shfl_xor(int(best), o)));
    const int v = 1023 - int(best & 1023u);
    int c = 0;
    for (int w = 0; w < 4; ++w) {
      const uint64_t free_bits = ~mask[v][w];
      if (free_bits) {
        c = w * 64 + __builtin_ctzll(free_bits);
        break;
      }
    }
    maxc = max(maxc, c + 1);
    __syncthreads();  // every lane has read this step's state
    if (lane == 0) col[v] = int16_t(c);
    const uint64_t bit = uint64_t(1) << (c & 63);
    for (int k = lptr[v0 + v] + lane; k < lptr[v0 + v + 1]; k += 64) {
      const int u = ladj[k] - v0;  // distinct neighbours: no two lanes share a row
      if (col[u] < 0 && !(mask[u][c >> 6] & bit)) {
        mask[u][c >> 6] |= bit;
        sat[u] = int16_t(sat[u] + 1);
      }
    }
    __syncthreads();
  }
  for (int v = lane; v < n; v += 64) lc[v0 + v] = col[v];
  if (lane == 0) pnlc[p] = maxc;
}

// Device buffers freed on scope exit (setup-time allocations only).
struct Scratch {
  std::vector<void*> p;
  template <typename T>
  T* get(size_t n) {
    T* q = dalloc<T>(n);
    p.push_back(q);
    return q;
  }
  template <typename T>
  T* up(const T* h, size_t n, hipStream_t st) {
    T* q = get<T>(n);
    if (n) HIPCHECK(hipMemcpyAsync(q, h, n * sizeof(T), hipMemcpyHostToDevice, st));
    return q;
  }
  ~Scratch() {
    for (void* q : p) (void)hipFree(q);
  }
};

unsigned blocks_for(int64_t n, int tpb) { return unsigned((n + tpb - 1) / tpb); }

}  // namespace

void knn_device(const double* queries, int64_t nq, const double* data, int64_t nd, int k, std::vector<int32_t>& idx,
                std::vector<double>& d2, hipStream_t st) {
  if (k < 1 || k > nd) throw Error(MGM_E_ARG, "knn: k out of range");
  if (k > 128) throw Error(MGM_E_ARG, "device knn: k must be <= 128");
  const KnnGrid g = knn_grid(data, nd, k);
  std::vector<double> sx(3 * size_t(nd));
  for (int64_t s = 0; s < nd; ++s)
    for (int a = 0; a < 3; ++a) sx[3 * s + a] = data[3 * size_t(g.pts[s]) + a];
  // queries in cell order (counting sort on the same grid)
  std::vector<int64_t> qcell(nq);
  std::vector<int32_t> qstart(g.start.size(), 0), qord(nq);
  for (int64_t q = 0; q < nq; ++q) {
    qcell[q] = g.cell_index(g.coord(queries[3 * q], 0), g.coord(queries[3 * q + 1], 1), g.coord(queries[3 * q + 2], 2));
    qstart[qcell[q] + 1]++;
  }
  for (size_t c = 0; c + 1 < qstart.size(); ++c) qstart[c + 1] += qstart[c];
  for (int64_t q = 0; q < nq; ++q) qord[qstart[qcell[q]]++] = int32_t(q);
  GridDev gd;
  for (int a = 0; a < 3; ++a) {
    gd.lo[a] = g.lo[a];
    gd.dim[a] = g.dim[a];
  }
  gd.h = g.h;
  Scratch s;
  const int32_t* d_ord = s.up(qord.data(), qord.size(), st);
  const double* d_q = s.up(queries, 3 * size_t(nq), st);
  const double* d_s = s.up(sx.data(), sx.size(), st);
  const int32_t* d_pts = s.up(g.pts.data(), g.pts.size(), st);
  const int32_t* d_start = s.up(g.start.data(), g.start.size(), st);
  int32_t* d_idx = s.get<int32_t>(size_t(nq) * k);
  double* d_d2 = s.get<double>(size_t(nq) * k);
  if (k <= 64)
    hipLaunchKernelGGL((k_knn<64, 64>), dim3(blocks_for(nq, 64)), dim3(64), 0, st, nq, k, d_ord, d_q, d_s, d_pts,
                       d_start, gd, d_idx, d_d2);
  else
    hipLaunchKernelGGL((k_knn<128, 32>), dim3(blocks_for(nq, 32)), dim3(32), 0, st, nq, k, d_ord, d_q, d_s, d_pts,
                       d_start, gd, d_idx, d_d2);
  HIPCHECK(hipGetLastError());
  idx.resize(size_t(nq) * k);
  d2.resize(size_t(nq) * k);
  HIPCHECK(hipMemcpyAsync(idx.data(), d_idx, idx.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(d2.data(), d_d2, d2.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
}

void dsatur_patches_device(const std::vector<int32_t>& lptr, const std::vector<int32_t>& ladj,
                           const std::vector<int32_t>& pstart, std::vector<int32_t>& lc, std::vector<int32_t>& pnlc,
                           hipStream_t st) {
  const int32_t np = int32_t(pstart.size()) - 1;
  for (int32_t p = 0; p < np; ++p)
    if (pstart[p + 1] - pstart[p] > kDsaturRows) throw Error(MGM_E_ARG, "device DSATUR: patch larger than 256 rows");
  const int32_t n = pstart.back();
  lc.assign(n, -1);
  pnlc.assign(np, 0);
  if (np == 0) return;
  Scratch s;
  const int32_t* d_ps = s.up(pstart.data(), pstart.size(), st);
  const int32_t* d_lptr = s.up(lptr.data(), lptr.size(), st);
  const int32_t* d_ladj = s.up(ladj.data(), ladj.size(), st);
  int32_t* d_lc = s.get<int32_t>(n);
  int32_t* d_pn = s.get<int32_t>(np);
  hipLaunchKernelGGL(k_dsatur, dim3(np), dim3(64), 0, st, d_ps, d_lptr, d_ladj, d_lc, d_pn);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(lc.data(), d_lc, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(pnlc.data(), d_pn, sizeof(int32_t) * np, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
}

Csr spgemm_device(const Csr& A, const Csr& B, hipStream_t st) {
  if (A.ncols != B.nrows) throw Error(MGM_E_ARG, "spgemm: inner dimensions differ");
  const int32_t n = A.nrows;
  Csr C;
  C.nrows = n;
  C.ncols = B.ncols;
  C.ptr.assign(n + 1, 0);
  if (n == 0) return C;
  Scratch s;
  const int32_t* aptr = s.up(A.ptr.data(), A.ptr.size(), st);
  const int32_t* acol = s.up(A.col.data(), A.col.size(), st);
  const double* aval = s.up(A.val.data(), A.val.size(), st);
  const int32_t* bptr = s.up(B.ptr.data(), B.ptr.size(), st);
  const int32_t* bcol = s.up(B.col.data(), B.col.size(), st);
  const double* bval = s.up(B.val.data(), B.val.size(), st);
  int64_t* cnt = s.get<int64_t>(n);
  hipLaunchKernelGGL(k_spgemm_count, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, aptr, acol, bptr, cnt);
  HIPCHECK(hipGetLastError());
  std::vector<int64_t> hcnt(n), hoff(n);
  HIPCHECK(hipMemcpyAsync(hcnt.data(), cnt, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  int64_t m = 0;
  for (int32_t i = 0; i < n; ++i) {
    hoff[i] = m;
    m += hcnt[i];
  }
  if (m == 0) return C;
  const int64_t* off = s.up(hoff.data(), hoff.size(), st);
  uint64_t* key0 = s.get<uint64_t>(m);
  uint64_t* key1 = s.get<uint64_t>(m);
  double* val0 = s.get<double>(m);
  double* val1 = s.get<double>(m);
  hipLaunchKernelGGL(k_spgemm_expand, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, aptr, acol, aval, bptr, bcol,
                     bval, off, key0, val0);
  HIPCHECK(hipGetLastError());
  // stable sort by (row, column): equal keys keep the expansion order
  int end_bit = 32;
  while (end_bit < 64 && (uint64_t(n - 1) >> (end_bit - 32)) != 0) ++end_bit;
  size_t tmp_bytes = 0;
  HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key0, key1, val0, val1, m, 0, end_bit, st));
  void* tmp = s.get<char>(tmp_bytes);
  HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key0, key1, val0, val1, m, 0, end_bit, st));
  int32_t* flag = s.get<int32_t>(m);
  int32_t* incl = s.get<int32_t>(m);
  hipLaunchKernelGGL(k_run_flags, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, key1, flag);
  HIPCHECK(hipGetLastError());
  size_t scan_bytes = 0;
  HIPCHECK(hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, flag, incl, m, st));
  void* stmp = s.get<char>(scan_bytes);
  HIPCHECK(hipcub::DeviceScan::InclusiveSum(stmp, scan_bytes, flag, incl, m, st));
  int32_t nruns32 = 0;
  HIPCHECK(hipMemcpyAsync(&nruns32, incl + (m - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  const int64_t nruns = nruns32;
  int64_t* heads = s.get<int64_t>(nruns);
  hipLaunchKernelGGL(k_heads, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, flag, incl, heads);
  int32_t* rrow = s.get<int32_t>(nruns);
  int32_t* rcol = s.get<int32_t>(nruns);
  double* rval = s.get<double>(nruns);
  hipLaunchKernelGGL(k_run_sums, dim3(blocks_for(nruns, 256)), dim3(256), 0, st, m, nruns, heads, key1, val1, rrow,
                     rcol, rval);
  HIPCHECK(hipGetLastError());
  std::vector<int32_t> hrow(nruns);
  C.col.resize(nruns);
  C.val.resize(nruns);
  HIPCHECK(hipMemcpyAsync(hrow.data(), rrow, sizeof(int32_t) * nruns, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(C.col.data(), rcol, sizeof(int32_t) * nruns, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(C.val.data(), rval, sizeof(double) * nruns, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  for (int64_t r = 0; r < nruns; ++r) C.ptr[hrow[r] + 1]++;
  for (int32_t i = 0; i < n; ++i) C.ptr[i + 1] += C.ptr[i];
  return C;
}

}  // namespace mgm
