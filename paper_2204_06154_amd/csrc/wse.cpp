// Weighted sample elimination (host), used to coarsen each point cloud
// (Sec. 4.1; Alg. 2). The coarse cloud keeps M = floor(N/factor) of the N
// points. Constants (the paper cites the method without them):
//   dbar   = mean nearest-other-point distance, summed in index order;
//   r_max  = dbar * sqrt(N / (4 M))   (2-D maximal Poisson-disk radius of M
//            points on an area N (sqrt 3/2) dbar^2);
//   pairs  = all i != j with d_ij < 2 r_max, d_ij = sqrt(d2_ij);
//   w(d)   = t^8, t = 1 - d/(2 r_max), by repeated squaring;
//   W_i    = sum of w over i's neighbours in ascending neighbour index.
// Then N - M times: eliminate the point with the largest W (ties: smaller
// index) and subtract its pair weight from each remaining neighbour in
// ascending neighbour index. Survivors are returned in ascending index.
// Compiled with -ffp-contract=off so the float sequence is reproducible.
#include <algorithm>
#include <cmath>
#include <queue>

#include "host_common.h"

namespace mgm {

std::vector<int32_t> wse_eliminate(const double* xyz, int64_t n, int factor) {
  const int64_t M = n / factor;
  if (M < 1 || n < 2) throw Error(MGM_E_ARG, "wse: too few points");
  std::vector<int32_t> nn;
  std::vector<double> nd2;
  knn_search(xyz, n, xyz, n, 2, nn, nd2);
  double sum = 0.0;
  for (int64_t i = 0; i < n; ++i) sum += std::sqrt(nd2[2 * i + 1]);
  const double dbar = sum / double(n);
  const double r_max = dbar * std::sqrt(double(n) / (4.0 * double(M)));
  const double two_r = 2.0 * r_max;

  // neighbour lists on a grid of cell size 2 r_max (27-cell search)
  double lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], xyz[3 * i + a]);
      hi[a] = std::max(hi[a], xyz[3 * i + a]);
    }
  double h = two_r;
  int dim[3];
  for (;;) {
    int64_t nc = 1;
    for (int a = 0; a < 3; ++a) {
      dim[a] = int((hi[a] - lo[a]) / h) + 1;
      nc *= dim[a];
    }
    if (nc <= (int64_t(1) << 24)) break;
    h *= 1.25;
  }
  auto cc = [&](double x, int a) {
    int t = int(std::floor((x - lo[a]) / h));
    return std::min(std::max(t, 0), dim[a] - 1);
  };
  int64_t ncell = int64_t(dim[0]) * dim[1] * dim[2];
  std::vector<int32_t> cstart(ncell + 1, 0), cpts(n);
  std::vector<int64_t> cell(n);
  for (int64_t i = 0; i < n; ++i) {
    cell[i] = (int64_t(cc(xyz[3 * i + 2], 2)) * dim[1] + cc(xyz[3 * i + 1], 1)) * dim[0] + cc(xyz[3 * i], 0);
    cstart[cell[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  {
    std::vector<int32_t> f(cstart.begin(), cstart.end() - 1);
    for (int64_t i = 0; i < n; ++i) cpts[f[cell[i]]++] = int32_t(i);
  }
  // per-point sorted neighbour lists with weights
  std::vector<std::vector<std::pair<int32_t, double>>> nb(n);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int c0 = cc(xyz[3 * i], 0), c1 = cc(xyz[3 * i + 1], 1), c2 = cc(xyz[3 * i + 2], 2);
      auto& L = nb[i];
      for (int z = std::max(0, c2 - 1); z <= std::min(dim[2] - 1, c2 + 1); ++z)
        for (int y = std::max(0, c1 - 1); y <= std::min(dim[1] - 1, c1 + 1); ++y)
          for (int x = std::max(0, c0 - 1); x <= std::min(dim[0] - 1, c0 + 1); ++x) {
            int64_t ci = (int64_t(z) * dim[1] + y) * dim[0] + x;
            for (int32_t t = cstart[ci]; t < cstart[ci + 1]; ++t) {
              int32_t j = cpts[t];
              if (j == i) continue;
              double dx = xyz[3 * j] - xyz[3 * i];
              double dy = xyz[3 * j + 1] - xyz[3 * i + 1];
              double dz = xyz[3 * j + 2] - xyz[3 * i + 2];
              double d = std::sqrt((dx * dx + dy * dy) + dz * dz);
              if (d < two_r) {
                double tt = 1.0 - d / two_r;
                double t2 = tt * tt;
                double t4 = t2 * t2;
                L.push_back({j, t4 * t4});
              }
            }
          }
      std::sort(L.begin(), L.end(), [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
        return a.first < b.first;
      });
    }
  });
  std::vector<double> W(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (auto& q : nb[i]) acc += q.second;
    W[i] = acc;
  }
  // max-heap on (W, -index) with lazy deletion
  struct Item {
    double w;
    int32_t i;
  };
  auto cmp = [](const Item& a, const Item& b) { return a.w < b.w || (a.w == b.w && a.i > b.i); };
  std::priority_queue<Item, std::vector<Item>, decltype(cmp)> heap(cmp);
  for (int64_t i = 0; i < n; ++i) heap.push({W[i], int32_t(i)});
  std::vector<char> removed(n, 0);
  for (int64_t t = 0; t < n - M; ++t) {
    Item it;
    for (;;) {
      it = heap.top();
      heap.pop();
      if (!removed[it.i] && it.w == W[it.i]) break;
    }
    removed[it.i] = 1;
    for (auto& q : nb[it.i]) {
      if (removed[q.first]) continue;
      W[q.first] = W[q.first] - q.second;
      heap.push({W[q.first], q.first});
    }
  }
  std::vector<int32_t> keep;
  keep.reserve(M);
  for (int64_t i = 0; i < n; ++i)
    if (!removed[i]) keep.push_back(int32_t(i));
  return keep;
}

}  // namespace mgm
