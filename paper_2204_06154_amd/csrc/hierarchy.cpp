// Preprocessing phase of MGM (Alg. 2), host side, FP64.
//
// Levels: N_{j+1} = floor(N_j / factor); with N_min > 0 the count is
// p = floor(log(N_1/N_min)/log 4) + 1 (evaluated as an integer loop, so that
// N_min <= N_p < 4 N_min), otherwise coarsen while N_j > n_coarse_max.
// Per level: WSE survivors (Sec. 4.1), interpolation I_{j+1}^j (Sec. 3,
// eq. rbf_fd_interp: PHS r plus a constant on the m nearest coarse points, a
// survivor's own row being the exact injection), R_j = P_j^T, Galerkin
// L_{j+1} = R_j L_j P_j on the structural product pattern (eq. galerkin), the
// border b_{j+1} = b_j P_j (eq. gco_saddle_point), the smoother colouring and
// finally the dense inverse of the coarsest (bordered) operator (Sec. 4.3).
#include "hierarchy.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <tuple>

namespace mgm {

void validate_params(const mgm_params& p, int64_t n) {
  auto bad = [](const char* m) { throw Error(MGM_E_ARG, m); };
  if (n < 16 || n > (int64_t(1) << 30)) bad("number of points out of range");
  if (p.disc != MGM_RBFFD && p.disc != MGM_GFD) bad("disc");
  if (p.poly_degree < 0 || p.poly_degree > 8) bad("poly_degree must be 0..8");
  // the Laplacian of r^(2k+1) is (2k+1)^2 r^(2k-1): finite at the stencil centre only for k >= 1
  if (p.disc == MGM_RBFFD && (p.phs_order < 1 || p.phs_order > 8)) bad("phs_order must be 1..8");
  int L = (p.poly_degree + 1) * (p.poly_degree + 2) / 2;
  if (p.stencil_size < L || p.stencil_size > 128 || p.stencil_size > n) bad("stencil_size");
  if (p.disc == MGM_GFD && !(p.gfd_alpha > 0)) bad("gfd_alpha must be > 0");
  if (p.problem != MGM_SCREENED && p.problem != MGM_POISSON) bad("problem");
  if (p.problem == MGM_SCREENED && !(std::isfinite(p.mu) && p.mu != 0.0))
    bad("mu must be finite and non-zero for the screened problem");
  if (p.interp_size < 1 || p.interp_size > 16) bad("interp_size");
  if (p.coarsen_factor < 2) bad("coarsen_factor");
  if (p.n_min < 0 || p.n_coarse_max < 0 || (p.n_min == 0 && p.n_coarse_max == 0)) bad("n_min / n_coarse_max");
  if (p.nu1 < 0 || p.nu2 < 0 || p.nu1 > 8 || p.nu2 > 8) bad("nu1/nu2");
  if (p.precision < MGM_FP64 || p.precision > MGM_FP16) bad("precision");
  if (p.gs_block < 0 || p.gs_block > 256) bad("gs_block must be 0..256");
  if (p.gs_max_width < 1 || p.gs_max_width > kMaxPatchWidth) bad("gs_max_width must be 1..96");
  if (p.gs_flow < 0 || p.gs_flow > 2) bad("gs_flow must be 0, 1 or 2");
  if (p.cycle < MGM_CYCLE_V || p.cycle > MGM_CYCLE_F) bad("cycle");
}

std::vector<int32_t> level_sizes(int64_t n1, const mgm_params& p) {
  std::vector<int32_t> s{int32_t(n1)};
  const int64_t f = p.coarsen_factor;
  if (p.n_min > 0) {
    int pcount = 1;
    int64_t pw = f;
    while (int64_t(p.n_min) * pw <= n1) {
      ++pcount;
      pw *= f;
    }
    for (int j = 1; j < pcount; ++j) s.push_back(int32_t(s.back() / f));
  } else {
    while (s.back() > p.n_coarse_max) s.push_back(int32_t(s.back() / f));
  }
  return s;
}

Csr transpose(const Csr& A) {
  Csr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.ptr.assign(A.ncols + 1, 0);
  for (int64_t k = 0; k < A.nnz(); ++k) T.ptr[A.col[k] + 1]++;
  for (int32_t i = 0; i < A.ncols; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.nnz());
  T.val.resize(A.nnz());
  std::vector<int32_t> fill(T.ptr.begin(), T.ptr.end() - 1);
  for (int32_t i = 0; i < A.nrows; ++i)
    for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int32_t t = fill[A.col[k]]++;
      T.col[t] = i;
      T.val[t] = A.val[k];
    }
  return T;  // rows ascending => columns sorted within each row
}

Csr spgemm_host(const Csr& A, const Csr& B) {
  Csr C;
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  std::vector<std::vector<int32_t>> rc(A.nrows);
  std::vector<std::vector<double>> rv(A.nrows);
  parallel_for(A.nrows, [&](int64_t b, int64_t e) {
    std::vector<int32_t> mark(B.ncols, -1);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int32_t> touched;
    for (int64_t i = b; i < e; ++i) {
      touched.clear();
      for (int32_t ka = A.ptr[i]; ka < A.ptr[i + 1]; ++ka) {
        int32_t k = A.col[ka];
        double a = A.val[ka];
        for (int32_t kb = B.ptr[k]; kb < B.ptr[k + 1]; ++kb) {
          int32_t j = B.col[kb];
          if (mark[j] != int32_t(i)) {
            mark[j] = int32_t(i);
            acc[j] = 0.0;
            touched.push_back(j);
          }
          acc[j] += a * B.val[kb];
        }
      }
      std::sort(touched.begin(), touched.end());
      rc[i] = touched;
      rv[i].resize(touched.size());
      for (size_t t = 0; t < touched.size(); ++t) rv[i][t] = acc[touched[t]];
    }
  });
  C.ptr.assign(A.nrows + 1, 0);
  for (int32_t i = 0; i < A.nrows; ++i) C.ptr[i + 1] = C.ptr[i] + int32_t(rc[i].size());
  C.col.resize(C.ptr.back());
  C.val.resize(C.ptr.back());
  for (int32_t i = 0; i < A.nrows; ++i) {
    std::copy(rc[i].begin(), rc[i].end(), C.col.begin() + C.ptr[i]);
    std::copy(rv[i].begin(), rv[i].end(), C.val.begin() + C.ptr[i]);
  }
  return C;
}

namespace {

inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void build_interp(const HostLevel& fine, const std::vector<double>& cxyz, int m, const KnnFn& knn, HostLevel& out) {
  const int64_t n = fine.n;
  const int64_t nc = int64_t(cxyz.size() / 3);
  std::vector<double> d2;
  knn(fine.xyz.data(), n, cxyz.data(), nc, m, out.pidx, d2);
  out.pw.assign(size_t(n) * m, 0.0);
  out.injected.assign(n, 0);
  out.m = m;
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<double> M(size_t(m + 1) * (m + 1)), rhs(m + 1);
    std::vector<int> piv(m + 1);
    for (int64_t i = b; i < e; ++i) {
      const int32_t* ci = &out.pidx[size_t(i) * m];
      if (d2[size_t(i) * m] == 0.0) {
        out.injected[i] = 1;
        out.pw[size_t(i) * m] = 1.0;
        continue;
      }
      for (int p = 0; p < m; ++p) {
        for (int q = 0; q < m; ++q) {
          const double* yp = &cxyz[3 * size_t(ci[p])];
          const double* yq = &cxyz[3 * size_t(ci[q])];
          double dx = yq[0] - yp[0], dy = yq[1] - yp[1], dz = yq[2] - yp[2];
          M[p * (m + 1) + q] = std::sqrt((dx * dx + dy * dy) + dz * dz);
        }
        M[p * (m + 1) + m] = 1.0;
        M[m * (m + 1) + p] = 1.0;
        rhs[p] = std::sqrt(d2[size_t(i) * m + p]);
      }
      M[m * (m + 1) + m] = 0.0;
      rhs[m] = 1.0;
      if (!lu_factor(M.data(), m + 1, piv.data()))
        throw Error(MGM_E_STENCIL_SINGULAR, "interpolation system singular at node " + std::to_string(i));
      lu_solve(M.data(), m + 1, piv.data(), rhs.data());
      for (int p = 0; p < m; ++p) out.pw[size_t(i) * m + p] = rhs[p];
    }
  });
  // structural CSR of P: injection rows 1 entry, others m entries sorted by column
  Csr& P = out.P;
  P.nrows = int32_t(n);
  P.ncols = int32_t(nc);
  P.ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) P.ptr[i + 1] = P.ptr[i] + (out.injected[i] ? 1 : m);
  P.col.resize(P.ptr.back());
  P.val.resize(P.ptr.back());
  for (int64_t i = 0; i < n; ++i) {
    int cnt = out.injected[i] ? 1 : m;
    std::vector<std::pair<int32_t, double>> r(cnt);
    for (int t = 0; t < cnt; ++t) r[t] = {out.pidx[size_t(i) * m + t], out.pw[size_t(i) * m + t]};
    std::sort(r.begin(), r.end());
    for (int t = 0; t < cnt; ++t) {
      P.col[P.ptr[i] + t] = r[t].first;
      P.val[P.ptr[i] + t] = r[t].second;
    }
  }
  out.R = transpose(P);
}

}  // namespace

Csr galerkin_product(const Csr& R, const Csr& A, const Csr& P) { return spgemm_host(R, spgemm_host(A, P)); }

SetupBackend host_backend() { return SetupBackend{stencil_weights_host, knn_search, spgemm_host, dsatur_patches_host}; }

// Symmetrised adjacency of A without the diagonal (sorted rows): row i is the
// union of row i of A and of A^T (both sorted), merged without duplicates.
static void symmetric_adjacency(const Csr& A, std::vector<int32_t>& ptr, std::vector<int32_t>& adj) {
  const int32_t n = A.nrows;
  // pattern of A^T (rows ascending, so each of its rows is sorted)
  std::vector<int32_t> tptr(n + 1, 0), tcol(A.nnz());
  for (int64_t k = 0; k < A.nnz(); ++k) tptr[A.col[k] + 1]++;
  for (int32_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
  {
    std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) tcol[fill[A.col[k]]++] = i;
  }
  std::vector<int64_t> off(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) off[i + 1] = off[i] + (A.ptr[i + 1] - A.ptr[i]) + (tptr[i + 1] - tptr[i]);
  std::vector<int32_t> buf(off[n]), len(n);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int32_t ka = A.ptr[i], ea = A.ptr[i + 1], kt = tptr[i], et = tptr[i + 1];
      int32_t* out = buf.data() + off[i];
      int32_t cnt = 0, last = -1;
      while (ka < ea || kt < et) {
        int32_t c;
        if (kt >= et || (ka < ea && A.col[ka] <= tcol[kt])) c = A.col[ka++];
        else c = tcol[kt++];
        if (c == last || c == int32_t(i)) continue;
        out[cnt++] = c;
        last = c;
      }
      len[i] = cnt;
    }
  });
  ptr.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + len[i];
  adj.resize(ptr[n]);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) std::copy(buf.begin() + off[i], buf.begin() + off[i] + len[i], adj.begin() + ptr[i]);
  });
}

// Jones-Plassmann colouring with largest-degree-first priorities: rank by
// (degree descending, splitmix64(i) >> 32 ascending, i ascending); each round,
// every uncoloured node above all its uncoloured neighbours takes the smallest
// colour not used by a coloured neighbour.
static std::vector<int32_t> jp_colour(const std::vector<int32_t>& ptr, const std::vector<int32_t>& adj, int* ncolours) {
  const int32_t n = int32_t(ptr.size()) - 1;
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::vector<uint32_t> hsh(n);
  for (int32_t i = 0; i < n; ++i) hsh[i] = uint32_t(splitmix64(uint64_t(i)) >> 32);
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    int32_t da = ptr[a + 1] - ptr[a], db = ptr[b + 1] - ptr[b];
    if (da != db) return da > db;
    if (hsh[a] != hsh[b]) return hsh[a] < hsh[b];
    return a < b;
  });
  std::vector<int32_t> prio(n);
  for (int32_t t = 0; t < n; ++t) prio[order[t]] = n - 1 - t;
  std::vector<int32_t> colour(n, -1);
  std::vector<char> sel(n, 0);
  int32_t left = n;
  int maxc = 0;
  while (left > 0) {
    parallel_for(n, [&](int64_t b, int64_t e) {
      for (int64_t v = b; v < e; ++v) {
        sel[v] = 0;
        if (colour[v] >= 0) continue;
        bool top = true;
        for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k) {
          int32_t u = adj[k];
          if (colour[u] < 0 && prio[u] > prio[v]) {
            top = false;
            break;
          }
        }
        sel[v] = top;
      }
    });
    parallel_for(n, [&](int64_t b, int64_t e) {
      std::vector<char> used;
      for (int64_t v = b; v < e; ++v) {
        if (!sel[v]) continue;
        used.assign(ptr[v + 1] - ptr[v] + 2, 0);
        for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k) {
          int32_t c = colour[adj[k]];
          if (c >= 0 && c < int32_t(used.size())) used[c] = 1;
        }
        int c = 0;
        while (used[c]) ++c;
        colour[v] = c;  // neighbours selected this round are never adjacent
      }
    });
    for (int32_t v = 0; v < n; ++v)
      if (sel[v]) {
        --left;
        maxc = std::max(maxc, colour[v] + 1);
      }
  }
  *ncolours = maxc;
  return colour;
}

std::vector<int32_t> colour_graph(const Csr& A, int* ncolours) {
  std::vector<int32_t> ptr, adj;
  symmetric_adjacency(A, ptr, adj);
  return jp_colour(ptr, adj, ncolours);
}

static uint64_t spread21(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffull;
  v = (v | v << 16) & 0x1f0000ff0000ffull;
  v = (v | v << 8) & 0x100f00f00f00f00full;
  v = (v | v << 4) & 0x10c30c30c30c30c3ull;
  v = (v | v << 2) & 0x1249249249249249ull;
  return v;
}

// Points sorted by (3-D Morton key, index); coordinates quantised to 21 bits as
// floor((x - lo) / ext * (2^21 - 1)), ext the largest bounding-box extent.
std::vector<int32_t> morton_order(const double* xyz, int32_t n) {
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = xyz[a];
  for (int32_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], xyz[3 * i + a]);
      hi[a] = std::max(hi[a], xyz[3 * i + a]);
    }
  double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  if (!(ext > 0.0)) ext = 1.0;
  std::vector<uint64_t> key(n);
  for (int32_t i = 0; i < n; ++i) {
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) q[a] = uint64_t(std::min(2097151.0, std::floor((xyz[3 * i + a] - lo[a]) / ext * 2097151.0)));
    key[i] = spread21(q[0]) | (spread21(q[1]) << 1) | (spread21(q[2]) << 2);
  }
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b] || (key[a] == key[b] && a < b); });
  return order;
}

// DSATUR (Brelaz 1979) on the nodes [v0, v1) of a graph whose edges never
// leave that range: repeatedly colour the uncoloured node with the most
// distinct neighbour colours (saturation), ties by larger degree, then smaller
// index, with the smallest colour no neighbour has. Stale heap entries (an
// older saturation) are skipped when popped. Returns the number of colours.
static int dsatur_range(const std::vector<int32_t>& ptr, const std::vector<int32_t>& adj, int32_t v0, int32_t v1,
                        std::vector<int32_t>& colour) {
  using Key = std::tuple<int32_t, int32_t, int32_t>;  // (saturation, degree, -index): largest first
  std::priority_queue<Key> heap;
  std::vector<std::vector<int32_t>> seen(v1 - v0);  // sorted distinct neighbour colours
  for (int32_t v = v0; v < v1; ++v) {
    colour[v] = -1;
    heap.emplace(0, ptr[v + 1] - ptr[v], -v);
  }
  int maxc = 0;
  while (!heap.empty()) {
    auto [sat, deg, mv] = heap.top();
    heap.pop();
    const int32_t v = -mv;
    auto& sv = seen[v - v0];
    if (colour[v] >= 0 || sat != int32_t(sv.size())) continue;
    int32_t c = 0;
    for (int32_t x : sv) {  // sorted: the first gap is the smallest free colour
      if (x != c) break;
      ++c;
    }
    colour[v] = c;
    maxc = std::max(maxc, c + 1);
    for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k) {
      const int32_t u = adj[k];
      if (colour[u] >= 0) continue;
      auto& su = seen[u - v0];
      auto it = std::lower_bound(su.begin(), su.end(), c);
      if (it != su.end() && *it == c) continue;
      su.insert(it, c);
      heap.emplace(int32_t(su.size()), ptr[u + 1] - ptr[u], -u);
    }
  }
  return maxc;
}

// Recursive largest first (Leighton 1979): colour classes are filled one at a
// time. A class starts with the uncoloured node with the most uncoloured
// neighbours (ties: smaller index); the uncoloured neighbours of a member are
// excluded from the class; the class then repeatedly takes the eligible node
// with the most excluded neighbours (ties: fewer eligible neighbours, then
// smaller index). Neighbour counts are updated as nodes change state. O(n^2)
// per class: meant for the small patch graph. Returns the number of colours.
static int rlf_colour(const std::vector<int32_t>& ptr, const std::vector<int32_t>& adj, std::vector<int32_t>& colour) {
  const int32_t n = int32_t(ptr.size()) - 1;
  colour.assign(n, -1);
  std::vector<char> uncol(n, 1), elig(n);
  std::vector<int32_t> n_unc(n), n_elig(n), n_excl(n);
  for (int32_t v = 0; v < n; ++v) n_unc[v] = ptr[v + 1] - ptr[v];
  int32_t left = n, c = 0;
  while (left > 0) {
    for (int32_t v = 0; v < n; ++v) {
      elig[v] = uncol[v];
      n_elig[v] = n_unc[v];
      n_excl[v] = 0;
    }
    int32_t v = -1;
    for (int32_t x = 0; x < n; ++x)
      if (elig[x] && (v < 0 || n_unc[x] > n_unc[v])) v = x;
    while (v >= 0) {
      colour[v] = c;
      elig[v] = 0;
      uncol[v] = 0;
      --left;
      for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k) {
        --n_elig[adj[k]];
        --n_unc[adj[k]];
      }
      for (int32_t k = ptr[v]; k < ptr[v + 1]; ++k) {
        const int32_t u = adj[k];
        if (!elig[u]) continue;
        elig[u] = 0;  // excluded from this class
        for (int32_t q = ptr[u]; q < ptr[u + 1]; ++q) {
          --n_elig[adj[q]];
          ++n_excl[adj[q]];
        }
      }
      v = -1;
      for (int32_t x = 0; x < n; ++x) {
        if (!elig[x]) continue;
        if (v < 0 || n_excl[x] > n_excl[v] || (n_excl[x] == n_excl[v] && n_elig[x] < n_elig[v])) v = x;
      }
    }
    ++c;
  }
  return c;
}

// Patch id of every point by recursive coordinate bisection: a set of more
// than `block` points is sorted by (coordinate, index) along the axis of its
// largest bounding-box extent (first such axis on ties) and cut after the
// first floor(nb/2)*block points, nb = ceil(n/block); the first half is cut
// before the second and the final sets are numbered in that order, so every
// patch holds exactly `block` points except the last.
static int32_t rcb_patches(const double* xyz, int32_t n, int block, std::vector<int32_t>& patch) {
  patch.assign(n, 0);
  std::vector<int32_t> ids(n);
  std::iota(ids.begin(), ids.end(), 0);
  int32_t next = 0;
  std::vector<std::pair<int32_t, int32_t>> stack{{0, n}};  // [begin, end) ranges of ids
  while (!stack.empty()) {
    auto [b, e] = stack.back();
    stack.pop_back();
    if (e - b <= block) {
      for (int32_t t = b; t < e; ++t) patch[ids[t]] = next;
      ++next;
      continue;
    }
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = xyz[3 * size_t(ids[b]) + a];
    for (int32_t t = b; t < e; ++t)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], xyz[3 * size_t(ids[t]) + a]);
        hi[a] = std::max(hi[a], xyz[3 * size_t(ids[t]) + a]);
      }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
      if (hi[a] - lo[a] > hi[axis] - lo[axis]) axis = a;
    const int32_t cut = ((e - b + block - 1) / block / 2) * block;
    // only the set of the first `cut` points matters: select, do not sort
    std::nth_element(ids.begin() + b, ids.begin() + b + cut, ids.begin() + e, [&](int32_t i, int32_t j) {
      const double xi = xyz[3 * size_t(i) + axis], xj = xyz[3 * size_t(j) + axis];
      return xi < xj || (xi == xj && i < j);
    });
    stack.emplace_back(b + cut, e);
    stack.emplace_back(b, b + cut);
  }
  return next;
}

// Smoother colouring of one level: patch-blocked (block > 0 and every row at
// most max_width entries) or plain multicolour.
void dsatur_patches_host(const std::vector<int32_t>& lptr, const std::vector<int32_t>& ladj,
                         const std::vector<int32_t>& pstart, std::vector<int32_t>& lc, std::vector<int32_t>& pnlc) {
  const int32_t np = int32_t(pstart.size()) - 1;
  lc.assign(pstart.back(), -1);
  pnlc.assign(np, 0);
  parallel_for(np, [&](int64_t b, int64_t e) {
    for (int64_t p = b; p < e; ++p) pnlc[p] = dsatur_range(lptr, ladj, pstart[p], pstart[p + 1], lc);
  }, 2);
}

void smoother_colouring(HostLevel& l, int block, int max_width, const DsaturFn& dsatur) {
  int32_t maxw = 0;
  for (int32_t i = 0; i < l.n; ++i) maxw = std::max(maxw, l.L.ptr[i + 1] - l.L.ptr[i]);
  std::vector<int32_t> ptr, adj;
  symmetric_adjacency(l.L, ptr, adj);
  l.patched = block > 0 && maxw <= max_width;
  if (!l.patched) {
    l.colour = jp_colour(ptr, adj, &l.ncolours);
    return;
  }
  const int32_t n = l.n;
  l.morton = morton_order(l.xyz.data(), n);
  l.npatch = rcb_patches(l.xyz.data(), n, block, l.patch);
  // patch graph and intra-patch graph
  std::vector<std::vector<int32_t>> pn(l.npatch);
  std::vector<int32_t> iptr(n + 1, 0), iadj;
  iadj.reserve(adj.size());
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
      int32_t j = adj[k];
      if (l.patch[j] != l.patch[i]) pn[l.patch[i]].push_back(l.patch[j]);
      else iadj.push_back(j);
    }
    iptr[i + 1] = int32_t(iadj.size());
  }
  std::vector<int32_t> pptr(l.npatch + 1, 0), padj;
  for (int32_t p = 0; p < l.npatch; ++p) {
    auto& r = pn[p];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    pptr[p + 1] = pptr[p] + int32_t(r.size());
    padj.insert(padj.end(), r.begin(), r.end());
  }
  const int npc = rlf_colour(pptr, padj, l.pcolour);
  // DSATUR on the union of the patch graphs = DSATUR on every patch alone (a
  // choice in one patch never changes another's saturations): run them in
  // parallel over the rows of each patch, renumbered to be contiguous.
  std::vector<int32_t> byp(n), pstart(l.npatch + 1, 0);
  for (int32_t i = 0; i < n; ++i) pstart[l.patch[i] + 1]++;
  for (int32_t p = 0; p < l.npatch; ++p) pstart[p + 1] += pstart[p];
  {
    std::vector<int32_t> fill(pstart.begin(), pstart.end() - 1);
    for (int32_t i = 0; i < n; ++i) byp[fill[l.patch[i]]++] = i;  // ascending index within a patch
  }
  std::vector<int32_t> pos(n);
  for (int32_t t = 0; t < n; ++t) pos[byp[t]] = t;
  std::vector<int32_t> lptr(n + 1, 0), ladj(iadj.size());
  for (int32_t t = 0; t < n; ++t) lptr[t + 1] = lptr[t] + (iptr[byp[t] + 1] - iptr[byp[t]]);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t t = b; t < e; ++t) {
      const int32_t i = byp[t];
      int32_t o = lptr[t];
      for (int32_t k = iptr[i]; k < iptr[i + 1]; ++k) ladj[o++] = pos[iadj[k]];
    }
  });
  std::vector<int32_t> lc, pnlc;
  dsatur(lptr, ladj, pstart, lc, pnlc);
  l.lcolour.resize(n);
  for (int32_t t = 0; t < n; ++t) l.lcolour[byp[t]] = lc[t];
  int nlc = 0;
  for (int32_t p = 0; p < l.npatch; ++p) nlc = std::max(nlc, pnlc[p]);
  l.npcolours = npc;
  // composite colour pcolour * nlc + lcolour, relabelled densely in order
  std::vector<int64_t> comp(n), used;
  for (int32_t i = 0; i < n; ++i) comp[i] = int64_t(l.pcolour[l.patch[i]]) * nlc + l.lcolour[i];
  used = comp;
  std::sort(used.begin(), used.end());
  used.erase(std::unique(used.begin(), used.end()), used.end());
  l.colour.resize(n);
  for (int32_t i = 0; i < n; ++i) l.colour[i] = int32_t(std::lower_bound(used.begin(), used.end(), comp[i]) - used.begin());
  l.ncolours = int(used.size());
}

void build_hierarchy(const double* xyz, const double* nrm, int64_t n, const mgm_params& p,
                     const SetupBackend& be, HostHierarchy& H) {
  validate_params(p, n);
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i]) || !std::isfinite(nrm[i])) throw Error(MGM_E_NONFINITE, "non-finite point or normal");
  H.params = p;
  H.normals.assign(nrm, nrm + 3 * n);
  std::vector<int32_t> sizes = level_sizes(n, p);
  if (sizes.size() < 2 || sizes.back() < 1) throw Error(MGM_E_ARG, "need at least two levels");
  const int ns = p.stencil_size;
  H.ns = ns;
  std::vector<double> d2;
  be.knn(xyz, n, xyz, n, ns, H.stencils, d2);
  for (int64_t i = 0; i < n; ++i) {
    if (ns > 1 && d2[size_t(i) * ns + 1] == 0.0) throw Error(MGM_E_DUP_POINTS, "duplicate points in the point cloud");
    if (H.stencils[size_t(i) * ns] != i) throw Error(MGM_E_DUP_POINTS, "stencil centre is not first");
  }
  be.weights(xyz, nrm, n, H.stencils.data(), ns, p, H.weights);
  for (double w : H.weights)
    if (!std::isfinite(w)) throw Error(MGM_E_NONFINITE, "non-finite stencil weight");

  H.lv.clear();
  H.lv.emplace_back();
  HostLevel& l1 = H.lv[0];
  l1.n = int32_t(n);
  l1.xyz.assign(xyz, xyz + 3 * n);
  // L_1 = D (Poisson) or I - mu D (screened), rows sorted by column
  l1.L.nrows = l1.L.ncols = int32_t(n);
  l1.L.ptr.resize(n + 1);
  l1.L.col.resize(size_t(n) * ns);
  l1.L.val.resize(size_t(n) * ns);
  for (int64_t i = 0; i <= n; ++i) l1.L.ptr[i] = int32_t(i * ns);
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<std::pair<int32_t, double>> r(ns);
    for (int64_t i = b; i < e; ++i) {
      for (int t = 0; t < ns; ++t) {
        double c = H.weights[size_t(i) * ns + t];
        double v;
        if (p.problem == MGM_POISSON) v = c;
        else v = (t == 0) ? 1.0 - p.mu * c : -(p.mu * c);
        r[t] = {H.stencils[size_t(i) * ns + t], v};
      }
      std::sort(r.begin(), r.end());
      for (int t = 0; t < ns; ++t) {
        l1.L.col[size_t(i) * ns + t] = r[t].first;
        l1.L.val[size_t(i) * ns + t] = r[t].second;
      }
    }
  });
  if (p.problem == MGM_POISSON) l1.b.assign(n, 1.0);

  for (size_t j = 0; j + 1 < sizes.size(); ++j) {
    HostLevel& f = H.lv[j];
    f.coarse_idx = wse_eliminate(f.xyz.data(), f.n, p.coarsen_factor);
    if (int32_t(f.coarse_idx.size()) != sizes[j + 1]) throw Error(MGM_E_ARG, "coarsening size mismatch");
    HostLevel c;
    c.n = sizes[j + 1];
    c.xyz.resize(size_t(c.n) * 3);
    for (int32_t t = 0; t < c.n; ++t)
      for (int a = 0; a < 3; ++a) c.xyz[3 * size_t(t) + a] = f.xyz[3 * size_t(f.coarse_idx[t]) + a];
    build_interp(f, c.xyz, std::min(p.interp_size, int(c.n)), be.knn, f);
    c.L = be.spgemm(f.R, be.spgemm(f.L, f.P));
    if (!f.b.empty()) {
      c.b.assign(c.n, 0.0);
      for (int32_t i = 0; i < c.n; ++i) {
        double s = 0.0;
        for (int32_t k = f.R.ptr[i]; k < f.R.ptr[i + 1]; ++k) s += f.R.val[k] * f.b[f.R.col[k]];
        c.b[i] = s;
      }
    }
    H.lv.push_back(std::move(c));
  }
  // zero diagonals and colours
  for (size_t j = 0; j < H.lv.size(); ++j) {
    HostLevel& l = H.lv[j];
    for (int32_t i = 0; i < l.n; ++i) {
      double d = 0.0;
      for (int32_t k = l.L.ptr[i]; k < l.L.ptr[i + 1]; ++k)
        if (l.L.col[k] == i) d = l.L.val[k];
      if (d == 0.0 && j + 1 < H.lv.size())
        throw Error(MGM_E_ZERO_DIAG, "zero diagonal on level " + std::to_string(j) + " row " + std::to_string(i));
    }
    if (j + 1 < H.lv.size()) smoother_colouring(l, p.gs_block, p.gs_max_width, be.dsatur);
  }
  // dense inverse of the coarsest (bordered) operator
  HostLevel& cl = H.lv.back();
  const int np = cl.n;
  const bool bord = p.problem == MGM_POISSON;
  const int dim = np + (bord ? 1 : 0);
  std::vector<double> A(size_t(dim) * dim, 0.0);
  for (int32_t i = 0; i < np; ++i)
    for (int32_t k = cl.L.ptr[i]; k < cl.L.ptr[i + 1]; ++k) A[size_t(i) * dim + cl.L.col[k]] = cl.L.val[k];
  if (bord)
    for (int32_t i = 0; i < np; ++i) {
      A[size_t(i) * dim + np] = cl.b[i];
      A[size_t(np) * dim + i] = cl.b[i];
    }
  std::vector<int> piv(dim);
  if (!lu_factor(A.data(), dim, piv.data())) throw Error(MGM_E_COARSE_SINGULAR, "coarsest operator is singular");
  H.coarse_dim = dim;
  H.coarse_inv.assign(size_t(dim) * dim, 0.0);
  parallel_for(dim, [&](int64_t b, int64_t e) {
    std::vector<double> x(dim);
    for (int64_t c = b; c < e; ++c) {
      std::fill(x.begin(), x.end(), 0.0);
      x[c] = 1.0;
      lu_solve(A.data(), dim, piv.data(), x.data());
      for (int r = 0; r < dim; ++r) H.coarse_inv[size_t(r) * dim + c] = x[r];
    }
  }, 64);
}

}  // namespace mgm
