// Surface gradient and divergence on the device (the operators of the heat
// method for geodesic distance, Sec. 6.3): tangent-plane RBF-FD weights, a
// vector W_ij per stencil entry, so that grad u(x_i) = sum_j W_ij u_j and
// div v(x_i) = sum_j W_ij . v_j. Both are HBM-bound stencil sweeps: one thread
// per node over entry-major (ns x N) weight planes and columns, so the lanes
// of a wavefront read consecutive addresses; the gathered u_j / v_j come
// mostly from the caches (stencils are spatially local).
#include <hip/hip_runtime.h>

#include "ctx.h"

namespace mgm {
namespace {

// g_i = sum_j W_ij u_j (N x 3, row-major); NORMALISE: g_i <- -g_i / |g_i|,
// the heat-method direction (0 where g_i = 0).
template <bool NORMALISE>
__global__ void k_surface_grad(int n, int ns, const int32_t* __restrict__ col, const double* __restrict__ w,
                               const double* __restrict__ u, double* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t plane = int64_t(ns) * n;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int t = 0; t < ns; ++t) {
    const int64_t e = int64_t(t) * n + i;
    const double uj = u[col[e]];
    gx += w[e] * uj;
    gy += w[plane + e] * uj;
    gz += w[2 * plane + e] * uj;
  }
  if (NORMALISE) {
    const double nrm = sqrt((gx * gx + gy * gy) + gz * gz);
    const double s = nrm > 0.0 ? -1.0 / nrm : 0.0;
    gx *= s;
    gy *= s;
    gz *= s;
  }
  g[3 * int64_t(i)] = gx;
  g[3 * int64_t(i) + 1] = gy;
  g[3 * int64_t(i) + 2] = gz;
}

// out_i = sum_j W_ij . v_j for a field v given as N x 3 (row-major).
__global__ void k_surface_div(int n, int ns, const int32_t* __restrict__ col, const double* __restrict__ w,
                              const double* __restrict__ v, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t plane = int64_t(ns) * n;
  double acc = 0.0;
  for (int t = 0; t < ns; ++t) {
    const int64_t e = int64_t(t) * n + i;
    const int64_t j = col[e];
    acc += (w[e] * v[3 * j] + w[plane + e] * v[3 * j + 1]) + w[2 * plane + e] * v[3 * j + 2];
  }
  out[i] = acc;
}

void need_surface_ops(const mgm_ctx* c) {
  need_device(c);
  if (!c->sg_wd) throw Error(MGM_E_ARG, "surface operators not set up (mgm_surface_ops_setup)");
}

}  // namespace
}  // namespace mgm

using namespace mgm;

extern "C" {

mgm_status mgm_surface_ops_setup(mgm_handle h, int32_t phs_order, int32_t poly_degree, int32_t stencil_size,
                                 void* stream) {
  if (!h) return MGM_E_ARG;
  return guard([&] {
    const int64_t n = h->H.lv[0].n;
    const int L = (poly_degree + 1) * (poly_degree + 2) / 2;
    if (poly_degree < 1 || poly_degree > 6 || phs_order < 1 || phs_order > 6 || stencil_size < L ||
        stencil_size > 128 || stencil_size > n)
      throw Error(MGM_E_ARG, "surface operators: need 1 <= poly_degree <= 6, 1 <= phs_order <= 6, "
                             "(l+1)(l+2)/2 <= stencil_size <= min(128, N)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool dev = h->device >= 0;
    if (dev) HIPCHECK(hipSetDevice(h->device));
    const double* xyz = h->H.lv[0].xyz.data();
    std::vector<int32_t> sten;
    std::vector<double> d2;
    if (dev && h->p.device_setup) knn_device(xyz, n, xyz, n, stencil_size, sten, d2, st);
    else knn_search(xyz, n, xyz, n, stencil_size, sten, d2);
    std::vector<double> W;
    surface_gradient_weights_host(xyz, h->H.normals.data(), n, sten.data(), stencil_size, phs_order, poly_degree, W);
    for (double v : W)
      if (!std::isfinite(v)) throw Error(MGM_E_NONFINITE, "non-finite gradient weight");
    const int ns = stencil_size;
    h->sg_ns = ns;
    h->sg_sten.swap(sten);
    h->sg_w.swap(W);
    if (!dev) return;  // host-only handle: weights for export only
    const std::vector<int32_t>& sg = h->sg_sten;
    const std::vector<double>& sw = h->sg_w;
    std::vector<int32_t> colp(size_t(ns) * n);
    std::vector<double> wp(size_t(3) * ns * n);
    for (int64_t i = 0; i < n; ++i)
      for (int t = 0; t < ns; ++t) {
        colp[size_t(t) * n + i] = sg[size_t(i) * ns + t];
        for (int a = 0; a < 3; ++a) wp[(size_t(a) * ns + t) * n + i] = sw[(size_t(i) * ns + t) * 3 + a];
      }
    h->sg_col = track(h, dupload(colp));
    h->sg_wd = track(h, dupload(wp));
  });
}

mgm_status mgm_surface_gradient(mgm_handle h, const double* d_u, double* d_g, int32_t normalise, void* stream) {
  if (!h || !d_u || !d_g) return MGM_E_ARG;
  return guard([&] {
    need_surface_ops(h);
    const int n = h->lv[0].n;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned g = unsigned((n + 255) / 256);
    if (normalise)
      hipLaunchKernelGGL(k_surface_grad<true>, dim3(g), dim3(256), 0, st, n, h->sg_ns, h->sg_col, h->sg_wd, d_u, d_g);
    else
      hipLaunchKernelGGL(k_surface_grad<false>, dim3(g), dim3(256), 0, st, n, h->sg_ns, h->sg_col, h->sg_wd, d_u, d_g);
    HIPCHECK(hipGetLastError());
  });
}

mgm_status mgm_surface_divergence(mgm_handle h, const double* d_v, double* d_out, void* stream) {
  if (!h || !d_v || !d_out) return MGM_E_ARG;
  return guard([&] {
    need_surface_ops(h);
    const int n = h->lv[0].n;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_surface_div, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, n, h->sg_ns, h->sg_col,
                       h->sg_wd, d_v, d_out);
    HIPCHECK(hipGetLastError());
  });
}

}  // extern "C"
