// Internal host-side types of the MGM library (not part of the C ABI).
#pragma once

#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mgm.h"

namespace mgm {

// Exception carrying an mgm_status; converted to a status code at the ABI.
struct Error : std::runtime_error {
  mgm_status status;
  Error(mgm_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

// Static partition of [0, n) over hardware threads (deterministic results:
// every index is processed by exactly one thread and no reductions cross
// threads).
inline int num_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 1;
  if (h > 32) h = 32;
  return int(h);
}

// Runs on one thread when n < min_items (small loops of cheap items); loops
// over few expensive items (patches, matrix columns) pass a smaller bound.
inline void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body, int64_t min_items = 2048) {
  int nt = num_threads();
  if (n < min_items || nt == 1) {
    body(0, n);
    return;
  }
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> errs(nt);
  int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([&, t, b, e] {
      try {
        body(b, e);
      } catch (...) {
        errs[t] = std::current_exception();
      }
    });
  }
  for (auto& x : th) x.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

// Compressed sparse rows, 32-bit indices, columns sorted within each row.
struct Csr {
  int32_t nrows = 0, ncols = 0;
  std::vector<int32_t> ptr, col;
  std::vector<double> val;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

// Dense grid of cubic cells over the bounding box of a point set, sized for
// k-nearest-neighbour searches; points bucketed by cell, ascending index
// within a cell.
struct KnnGrid {
  double lo[3], h;
  int dim[3];
  std::vector<int32_t> start;  // ncells + 1
  std::vector<int32_t> pts;    // point indices sorted by cell, then index
  int64_t cell_index(int cx, int cy, int cz) const;
  int coord(double x, int a) const;  // clamped cell coordinate along axis a
};
KnnGrid knn_grid(const double* data, int64_t nd, int k);

// kNN under the key (d2, index), d2 = ((dx*dx) + (dy*dy)) + dz*dz.
// queries: nq x 3, data: nd x 3 (row-major). Outputs nq x k indices / d2.
void knn_search(const double* queries, int64_t nq, const double* data, int64_t nd, int k,
                std::vector<int32_t>& idx, std::vector<double>& d2);

// Tangent-plane stencil weights of the Laplace-Beltrami operator (Sec. 2).
void stencil_weights_host(const double* xyz, const double* nrm, int64_t n, const int32_t* sten,
                          int ns, const mgm_params& p, std::vector<double>& w);

// Tangent-plane RBF-FD surface gradient weights, n x ns x 3 (W_ij, a vector
// per entry): grad u(x_i) = sum_j W_ij u_j, div v(x_i) = sum_j W_ij . v_j.
void surface_gradient_weights_host(const double* xyz, const double* nrm, int64_t n, const int32_t* sten, int ns,
                                   int phs_order, int deg, std::vector<double>& W);

// Tangent-plane coordinates (ns x 2) of the stencil st of node i (Sec. 2.1).
void project_stencil(const double* xyz, const double* nrm, int64_t i, const int32_t* st, int ns, double* xh);

// Survivor indices (ascending) of weighted sample elimination (Sec. 4.1).
std::vector<int32_t> wse_eliminate(const double* xyz, int64_t n, int factor);

// Jones-Plassmann largest-degree-first colouring of the symmetrised graph of A.
std::vector<int32_t> colour_graph(const Csr& A, int* ncolours);

// C = A * B on the structural product pattern, columns sorted per row; entry
// (i, j) is summed from 0.0 over the row of A in ascending column order.
Csr spgemm_host(const Csr& A, const Csr& B);
// C = R * A * P with the structural product pattern.
Csr galerkin_product(const Csr& R, const Csr& A, const Csr& P);
Csr transpose(const Csr& A);

// LU with partial pivoting (first maximal |pivot|), in place on a row-major
// n x n matrix; returns false if a pivot is exactly zero.
bool lu_factor(double* a, int n, int* piv);
void lu_solve(const double* lu, int n, const int* piv, double* x);

}  // namespace mgm
