// Host-side multilevel hierarchy built by the preprocessing phase (Alg. 2).
#pragma once

#include <functional>

#include "host_common.h"

namespace mgm {

struct HostLevel {
  int32_t n = 0;
  std::vector<double> xyz;            // n x 3
  Csr L;                              // L_j, natural numbering, structural pattern
  std::vector<double> b;              // border b_j (Poisson only)
  std::vector<int32_t> colour;        // smoother colour per row (all but the coarsest)
  int ncolours = 0;
  // patch-blocked smoother ordering (see smoother_colouring)
  bool patched = false;
  std::vector<int32_t> morton;        // points sorted by Morton key
  std::vector<int32_t> patch;         // patch of each row
  std::vector<int32_t> pcolour;       // colour of each patch
  std::vector<int32_t> lcolour;       // colour of each row inside its patch
  int32_t npatch = 0;
  int npcolours = 0;
  // transfer to level j+1 (all but the coarsest)
  std::vector<int32_t> coarse_idx;    // survivors of WSE, ascending level-j index
  int m = 0;                          // interpolation stencil size
  std::vector<int32_t> pidx;          // n x m coarse neighbours (level j+1 numbering)
  std::vector<double> pw;             // n x m weights (injection rows: 1, 0, ...)
  std::vector<char> injected;         // row is a survivor (injection)
  Csr P, R;
};

// Computes the N x ns fine-level stencil weights (host or device backend).
using WeightsFn = std::function<void(const double* xyz, const double* nrm, int64_t n, const int32_t* sten,
                                     int ns, const mgm_params& p, std::vector<double>& w)>;

struct HostHierarchy {
  mgm_params params{};
  std::vector<HostLevel> lv;
  int ns = 0;
  std::vector<int32_t> stencils;      // N_1 x ns, centre first
  std::vector<double> weights;        // N_1 x ns
  std::vector<double> normals;        // N_1 x 3 (as given)
  int coarse_dim = 0;                 // N_p (screened) or N_p + 1 (bordered)
  std::vector<double> coarse_inv;     // dense row-major inverse of the coarsest system
};

constexpr int kMaxPatchWidth = 96;   // rows longer than this disable patch blocking on a level

// k nearest neighbours of the queries among the data points (host or device).
using KnnFn = std::function<void(const double* queries, int64_t nq, const double* data, int64_t nd, int k,
                                 std::vector<int32_t>& idx, std::vector<double>& d2)>;
// C = A * B on the structural product pattern (host or device).
using SpgemmFn = std::function<Csr(const Csr& A, const Csr& B)>;
// DSATUR colouring of every patch's graph: rows numbered so that patch p holds
// [pstart[p], pstart[p+1]) and no edge (lptr, ladj) leaves its patch; writes
// each row's colour to lc and each patch's colour count to pnlc (host or device).
using DsaturFn = std::function<void(const std::vector<int32_t>& lptr, const std::vector<int32_t>& ladj,
                                    const std::vector<int32_t>& pstart, std::vector<int32_t>& lc,
                                    std::vector<int32_t>& pnlc)>;
void dsatur_patches_host(const std::vector<int32_t>& lptr, const std::vector<int32_t>& ladj,
                         const std::vector<int32_t>& pstart, std::vector<int32_t>& lc, std::vector<int32_t>& pnlc);

// The preprocessing steps that have a host and a device implementation; both
// give identical results.
struct SetupBackend {
  WeightsFn weights;
  KnnFn knn;
  SpgemmFn spgemm;
  DsaturFn dsatur;
};
SetupBackend host_backend();

void validate_params(const mgm_params& p, int64_t n);
std::vector<int32_t> level_sizes(int64_t n1, const mgm_params& p);
void build_hierarchy(const double* xyz, const double* nrm, int64_t n, const mgm_params& p,
                     const SetupBackend& be, HostHierarchy& H);

}  // namespace mgm
