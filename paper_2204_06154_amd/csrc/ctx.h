// Internal device-side context of the MGM library (shared by the HIP
// translation units; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "hierarchy.h"
#include "kernels.h"

namespace mgm {

void knn_device(const double* queries, int64_t nq, const double* data, int64_t nd, int k, std::vector<int32_t>& idx,
                std::vector<double>& d2, hipStream_t st);
Csr spgemm_device(const Csr& A, const Csr& B, hipStream_t st);
void dsatur_patches_device(const std::vector<int32_t>& lptr, const std::vector<int32_t>& ladj,
                           const std::vector<int32_t>& pstart, std::vector<int32_t>& lc, std::vector<int32_t>& pnlc,
                           hipStream_t st);
// mixed: FP32 elimination on the matrix cores with FP64 refinement
// (poly_degree <= 4) instead of the FP64 elimination
void batched_phs_weights_device(const double* d_xyz, const double* d_nrm, const int32_t* d_sten, int64_t nsys, int ns,
                                int phs_order, int deg, double* d_w, int* d_status, hipStream_t st, bool mixed = false);

#define HIPCHECK(x)                                                                                     \
  do {                                                                                                  \
    hipError_t e_ = (x);                                                                                \
    if (e_ != hipSuccess) throw Error(MGM_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));      \
  } while (0)

inline unsigned nblk(int64_t threads) { return unsigned((threads + kBlock - 1) / kBlock); }

template <typename T>
T* dalloc(size_t n) {
  T* p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(reinterpret_cast<void**>(&p), n * sizeof(T)) != hipSuccess)
    throw Error(MGM_E_ALLOC, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  return p;
}

template <typename T>
T* dupload(const std::vector<T>& v) {
  T* p = dalloc<T>(v.size());
  if (!v.empty()) HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

// IEEE binary16 (round to nearest, ties to even) of a double, rounded once.
inline uint16_t f64_to_f16_bits(double x) {
  uint16_t sign = std::signbit(x) ? 0x8000 : 0;
  double a = std::fabs(x);
  if (std::isnan(x)) return sign | 0x7e00;
  if (a == 0.0) return sign;
  int E;
  std::frexp(a, &E);  // a = f 2^E, f in [0.5, 1)
  int e = E - 1;      // a in [2^e, 2^(e+1))
  if (e < -14) {      // subnormal grid: multiples of 2^-24
    double k = std::rint(std::ldexp(a, 24));
    return sign | uint16_t(k);  // k == 1024 is the smallest normal, encoded the same way
  }
  double k = std::rint(std::ldexp(a, 10 - e));  // in [1024, 2048]
  if (k == 2048.0) {
    k = 1024.0;
    ++e;
  }
  if (e > 15) return sign | 0x7c00;
  return sign | uint16_t((e + 15) << 10) | uint16_t(int(k) - 1024);
}

struct DevLevel {
  int n = 0, ncol = 0, W = 0, G = 8, m = 0, nnext = 0;
  int64_t nnz = 0;
  std::vector<int> cstart;           // colour row ranges (host)
  int32_t* perm = nullptr;           // position -> natural index (null: identity)
  int32_t *rowptr = nullptr, *col = nullptr;
  double* v64 = nullptr;
  float* v32 = nullptr;
  _Float16* v16 = nullptr;
  float* s16 = nullptr;
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  float* dinv16 = nullptr;
  int32_t* pcol = nullptr;
  double* p64 = nullptr;
  float* p32 = nullptr;
  int32_t *rptr = nullptr, *rcol = nullptr;
  double* r64 = nullptr;
  float* r32 = nullptr;
  double* b64 = nullptr;
  float* b32 = nullptr;
  double *e64 = nullptr, *f64 = nullptr, *res64 = nullptr;
  float *e32 = nullptr, *f32 = nullptr, *res32 = nullptr;
  // host copies needed to build reduced-precision values lazily
  std::vector<double> hv, hdiag;
  std::vector<int64_t> rowlen_prefix;  // host copy of the permuted row pointer
  // patch-blocked smoother (see k_gs_patch)
  bool patched = false;
  int wmax = 0;                      // register width class of the patch kernels (24, 32, .., 96)
  std::vector<int> pc_start;         // slot range of each patch colour (host)
  std::vector<int64_t> pc_nnz;       // stored entries (incl. padding) per patch colour (host)
  std::vector<int32_t> pc_rows;      // rows per patch colour (host)
  int32_t *pstart = nullptr, *pncl = nullptr, *lcol = nullptr, *pcolidx = nullptr;
  int pw = 0, pblock = 0;  // patch ELL: entries per lane and rows per slot
  int pstart_host_slots = 0;  // number of patch slots
  double* pv64 = nullptr;
  float* pv32 = nullptr;
  _Float16* pv16 = nullptr;
  std::vector<double> hpv;           // host copy of the patch values (FP64)
  std::vector<int32_t> hprow;        // permuted row of each patch entry (host)
  // one-launch sweeps (see GsFlow): coupled slots, colour row ranges, sweep state
  bool flow_ok = false;
  int32_t *fl_nbptr = nullptr, *fl_nb = nullptr, *fl_crow = nullptr;
  unsigned long long* fl_ticket = nullptr;
  unsigned* fl_flag = nullptr;
  // staged halo of the one-launch sweeps (see kMaxHalo): columns in staged
  // form, per-slot lists of distinct out-of-patch rows
  bool halo_ok = false;
  int32_t *pcolh = nullptr, *fl_hstart = nullptr, *fl_hrows = nullptr;
};

}  // namespace mgm

namespace mgm {

// Learned smoother of one level: MLP parameters and Adam moments, features,
// step weights, training snapshots and scratch.
struct LearnedLevel {
  bool active = false;
  int s = 0, nin = 0, T = 0, adam_t = 0, steps_cap = 0;
  int snap_cap = 0;   // snapshots (and c_t) that snap / c hold
  size_t z_cap = 0;   // floats that z holds (snapshots x steps x rows)
  double lam = 0.0;
  std::vector<double> wcheb;
  double* wcheb_d = nullptr;
  float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  double* om64 = nullptr;
  float* om32 = nullptr;
  float *X = nullptr, *O = nullptr, *H1 = nullptr, *H2 = nullptr, *dO = nullptr, *dH1 = nullptr, *dH2 = nullptr,
        *domega = nullptr, *omt = nullptr;
  float *snap = nullptr, *z = nullptr, *e = nullptr, *y = nullptr, *g = nullptr, *t = nullptr;
  int32_t *tptr = nullptr, *tcol = nullptr;
  float* tval = nullptr;
  double *c = nullptr, *loss = nullptr, *scal = nullptr;
  float* atb = nullptr;
  double* atb2 = nullptr;  // group sums of the partials
};

}  // namespace mgm

struct mgm_ctx {
  int device = 0;
  mgm_params p{};
  mgm::HostHierarchy H;
  std::vector<mgm::DevLevel> lv;     // all levels; the last is the coarsest
  int cdim = 0;
  double* cinv = nullptr;
  double* rho = nullptr;             // per-level constraint residuals
  double* mu = nullptr;              // multiplier correction (bordered)
  double* lam = nullptr;             // scalar for level ops
  double* partial = nullptr;
  int64_t partial_len = 0;
  bool built[3] = {true, false, false};
  hipStream_t cap = nullptr;
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  std::vector<void*> allocs;
  // solver workspace
  int ws_restart = 0;
  int64_t ld = 0;
  double *V = nullptr, *Z = nullptr, *vecs = nullptr, *kpart = nullptr, *dh = nullptr;
  double* hpin = nullptr;  // pinned host copies of dot results
  int* flow_err = nullptr;   // device: a one-launch sweep gave up waiting
  int* hflow_err = nullptr;  // pinned host copy
  unsigned long long flow_wait_ticks = 0;  // bound of the one-launch sweeps' waits (set at setup)
  hipEvent_t step_done = nullptr;  // FGMRES: end of an Arnoldi step's kernels
  double* capture = nullptr;         // when set: the start level's vector after the coarse correction (eager cycle)
  int capture_level = 0;
  // learned smoothers, one state per smoothed level (see learned.hip)
  std::vector<mgm::LearnedLevel> ls;
  double* e_tmp64 = nullptr;         // ping-pong buffer of the Richardson steps (fine-level size)
  float* e_tmp32 = nullptr;
  // surface gradient / divergence operator (heat-method geodesics)
  int sg_ns = 0;
  std::vector<int32_t> sg_sten;      // N_1 x ns stencils (caller order)
  std::vector<double> sg_w;          // N_1 x ns x 3 weights W_ij
  int32_t* sg_col = nullptr;         // ns x N_1, entry-major
  double* sg_wd = nullptr;           // 3 planes of ns x N_1, entry-major
};

namespace mgm {

extern thread_local std::string g_last_error;

template <typename T>
inline T* track(mgm_ctx* c, T* p) {
  c->allocs.push_back(reinterpret_cast<void*>(p));
  return p;
}

// shared helpers of the HIP translation units (defined in device.hip)
void build_precision(mgm_ctx* c, int prec);
void vcycle_core(mgm_ctx* c, hipStream_t st);
void precond(mgm_ctx* c, const double* v, double* z, const int32_t* perm, hipStream_t st);
void apply_A(mgm_ctx* c, const double* x, double* y, hipStream_t st);
void ensure_ws(mgm_ctx* c, int restart);
void mdot(mgm_ctx* c, int64_t n, const double* V, int64_t ld, int k, const double* w, double* out, hipStream_t st,
          double* host_out = nullptr);
void host_wait(hipStream_t st);
void to_host(mgm_ctx* c, const double* d, int k, hipStream_t st);
// z = M_j v for FP64 vectors in level j's permuted order: the cycle of the
// sub-hierarchy that starts at level j (j >= 1), run eagerly in the handle's
// precision; bordered problems: n_j + 1 entries, the multiplier (constraint
// residual in v, multiplier correction in z) at index n_j.
void precond_level(mgm_ctx* c, int j, const double* v, double* z, hipStream_t st);
// y = A_j x, FP64, level j's permuted order: L_j, or bordered the level's
// [L_j b_j; b_j^T 0] on n_j + 1 entries.
void spmv_level64(mgm_ctx* c, int j, const double* x, double* y, hipStream_t st);
inline bool learned_on(const mgm_ctx* c, int j) { return j < int(c->ls.size()) && c->ls[j].active; }
void need_device(const mgm_ctx* c);
mgm_status guard(const std::function<void()>& f);
void invalidate_graphs(mgm_ctx* c);
// Waits for the stream; if a one-launch sweep gave up waiting since the last
// check, clears the error, resets every level's ticket counter and flags (so
// the next sweeps number from 1 again) and throws MGM_E_SYNC.
void flow_check(mgm_ctx* c, hipStream_t st);

}  // namespace mgm
