// Exact k-nearest-neighbour search on a uniform cell grid (host).
//
// Stencils are the n nearest points of the cloud to each centre under the
// Euclidean distance in R^3, centre included (Sec. 2); the interpolation uses
// the m nearest coarse points (Sec. 3). Ordering key: (d2, index) ascending
// with d2 = ((dx*dx) + (dy*dy)) + dz*dz in IEEE double, no contraction
// (this file is compiled with -ffp-contract=off), so the result is a unique,
// reproducible list even with exactly tied distances.
//
// Search: data points are bucketed in a dense grid of cubic cells; a query
// scans rings of cells of growing Chebyshev radius until the k-th best key is
// strictly inside the sphere that the scanned cube is guaranteed to contain.
#include <algorithm>
#include <cmath>
#include <limits>

#include "host_common.h"

namespace mgm {

int64_t KnnGrid::cell_index(int cx, int cy, int cz) const { return (int64_t(cz) * dim[1] + cy) * dim[0] + cx; }

int KnnGrid::coord(double x, int a) const {
  double t = std::floor((x - lo[a]) / h);
  if (!(t >= 0)) return 0;
  if (t >= dim[a] - 1) return dim[a] - 1;
  return int(t);
}

KnnGrid knn_grid(const double* data, int64_t nd, int k) {
  KnnGrid g;
  double hi[3];
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = std::numeric_limits<double>::infinity();
    hi[a] = -g.lo[a];
  }
  for (int64_t i = 0; i < nd; ++i)
    for (int a = 0; a < 3; ++a) {
      g.lo[a] = std::min(g.lo[a], data[3 * i + a]);
      hi[a] = std::max(hi[a], data[3 * i + a]);
    }
  double ext[3], vol = 1.0;
  for (int a = 0; a < 3; ++a) {
    ext[a] = std::max(hi[a] - g.lo[a], 1e-300);
    vol *= ext[a];
  }
  double maxext = std::max(ext[0], std::max(ext[1], ext[2]));
  // about max(k,8)/4 points per cell for volumetric data, more for surfaces
  double per = std::max(2.0, double(std::max(k, 8)) / 4.0);
  double h = std::cbrt(vol * per / double(std::max<int64_t>(nd, 1)));
  if (!(h > 0)) h = maxext;
  h = std::max(h, maxext / 1024.0);
  for (;;) {
    int64_t nc = 1;
    for (int a = 0; a < 3; ++a) nc *= int64_t(ext[a] / h) + 1;
    if (nc <= (int64_t(1) << 24)) break;
    h *= 1.25;
  }
  g.h = h;
  for (int a = 0; a < 3; ++a) g.dim[a] = int(ext[a] / h) + 1;
  int64_t ncells = int64_t(g.dim[0]) * g.dim[1] * g.dim[2];
  std::vector<int64_t> cell(nd);
  g.start.assign(ncells + 1, 0);
  for (int64_t i = 0; i < nd; ++i) {
    cell[i] = g.cell_index(g.coord(data[3 * i], 0), g.coord(data[3 * i + 1], 1),
                           g.coord(data[3 * i + 2], 2));
    g.start[cell[i] + 1]++;
  }
  for (int64_t c = 0; c < ncells; ++c) g.start[c + 1] += g.start[c];
  g.pts.resize(nd);
  std::vector<int32_t> fill(g.start.begin(), g.start.end() - 1);
  for (int64_t i = 0; i < nd; ++i) g.pts[fill[cell[i]]++] = int32_t(i);
  return g;
}

namespace {

struct Cand {
  double d2;
  int32_t j;
};
inline bool key_less(const Cand& a, const Cand& b) {
  return a.d2 < b.d2 || (a.d2 == b.d2 && a.j < b.j);
}

}  // namespace

void knn_search(const double* queries, int64_t nq, const double* data, int64_t nd, int k,
                std::vector<int32_t>& idx, std::vector<double>& d2out) {
  if (k < 1 || k > nd) throw Error(MGM_E_ARG, "knn: k out of range");
  KnnGrid g = knn_grid(data, nd, k);
  idx.assign(size_t(nq) * k, 0);
  d2out.assign(size_t(nq) * k, 0.0);
  const double inf = std::numeric_limits<double>::infinity();
  parallel_for(nq, [&](int64_t b, int64_t e) {
    std::vector<Cand> cand, tmp;
    for (int64_t q = b; q < e; ++q) {
      const double qx = queries[3 * q], qy = queries[3 * q + 1], qz = queries[3 * q + 2];
      int c[3] = {g.coord(qx, 0), g.coord(qy, 1), g.coord(qz, 2)};
      double qa[3] = {qx, qy, qz};
      cand.clear();
      for (int R = 0;; ++R) {
        bool covers_all = true;
        for (int a = 0; a < 3; ++a)
          if (c[a] - R > 0 || c[a] + R < g.dim[a] - 1) covers_all = false;
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::max(0, c[a] - R);
          hi[a] = std::min(g.dim[a] - 1, c[a] + R);
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
          for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
              int ring = std::max(std::abs(x - c[0]), std::max(std::abs(y - c[1]), std::abs(z - c[2])));
              if (ring != R) continue;
              int64_t ci = g.cell_index(x, y, z);
              for (int32_t t = g.start[ci]; t < g.start[ci + 1]; ++t) {
                int32_t j = g.pts[t];
                double dx = data[3 * j] - qx;
                double dy = data[3 * j + 1] - qy;
                double dz = data[3 * j + 2] - qz;
                double dd = (dx * dx + dy * dy) + dz * dz;
                cand.push_back({dd, j});
              }
            }
        if (int64_t(cand.size()) >= k) {
          tmp = cand;
          std::nth_element(tmp.begin(), tmp.begin() + (k - 1), tmp.end(), key_less);
          double kth = tmp[k - 1].d2;
          if (covers_all) break;
          double rcov = inf;
          for (int a = 0; a < 3; ++a) {
            if (c[a] - R > 0) rcov = std::min(rcov, qa[a] - (g.lo[a] + double(c[a] - R) * g.h));
            if (c[a] + R < g.dim[a] - 1) rcov = std::min(rcov, (g.lo[a] + double(c[a] + R + 1) * g.h) - qa[a]);
          }
          if (rcov == inf || kth < rcov * rcov * (1.0 - 1e-12)) break;
        } else if (covers_all) {
          break;
        }
      }
      std::partial_sort(cand.begin(), cand.begin() + k, cand.end(), key_less);
      for (int t = 0; t < k; ++t) {
        idx[size_t(q) * k + t] = cand[t].j;
        d2out[size_t(q) * k + t] = cand[t].d2;
      }
    }
  });
}

}  // namespace mgm
