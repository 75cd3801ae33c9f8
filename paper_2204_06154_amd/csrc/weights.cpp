// Tangent-plane stencil weights of the Laplace-Beltrami operator (host, FP64).
//
// Sec. 2.1 (eq. tp_pts): xh_j = Q^T (x_j - x_i), Q = [t1 t2] an orthonormal
// basis of the tangent plane at x_i. We take the coordinate axis e least
// aligned with the normal, t1 = normalise(e - (n.e) n), t2 = n x t1.
// Coordinates are scaled by s_i = max_j |xh_j| and the weights divided by s_i^2
// afterwards (both discretisations are scale-equivariant).
//
// RBF-FD (Sec. 2.2, eq. rbf_fd_lap): [A P; P^T 0][c; lambda] = [Lap phi; Lap p]
// with A_jk = |xi_j - xi_k|^(2k+1), P_jq = monomials by total degree then
// descending power of x, Lap r^m = m^2 r^(m-2) in 2-D, Lap p(0) = 2 for x^2
// and y^2. Solved by LU with partial pivoting (A has a zero diagonal).
//
// GFD (Sec. 2.3, eq. wls_fd_lap): weights w_j = exp(-alpha |xh_j|^2 /
// (rho_i^2 + rho_j^2)), rho_j the radius of node j's own projected stencil;
// c = W^{1/2} Q R^{-T} Lap p with W^{1/2} P = QR (Householder).
#include <algorithm>
#include <cmath>

#include "host_common.h"

namespace mgm {

bool lu_factor(double* a, int n, int* piv) {
  double amax = 0.0;
  for (int i = 0; i < n * n; ++i) amax = std::max(amax, std::fabs(a[i]));
  const double tiny = amax * 1e-13;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(a[k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::fabs(a[i * n + k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    piv[k] = p;
    if (!(best > tiny)) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(a[k * n + j], a[p * n + j]);
    const double inv = 1.0 / a[k * n + k];
    for (int i = k + 1; i < n; ++i) {
      double m = a[i * n + k] * inv;
      a[i * n + k] = m;
      if (m != 0.0) {
        const double* rk = a + k * n;
        double* ri = a + i * n;
        for (int j = k + 1; j < n; ++j) ri[j] -= m * rk[j];
      }
    }
  }
  return true;
}

void lu_solve(const double* lu, int n, const int* piv, double* x) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) std::swap(x[k], x[piv[k]]);
  for (int i = 1; i < n; ++i) {
    double s = x[i];
    for (int j = 0; j < i; ++j) s -= lu[i * n + j] * x[j];
    x[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int j = i + 1; j < n; ++j) s -= lu[i * n + j] * x[j];
    x[i] = s / lu[i * n + i];
  }
}

namespace {

void tangent_basis(const double* nrm, double t1[3], double t2[3]) {
  double nn = std::sqrt((nrm[0] * nrm[0] + nrm[1] * nrm[1]) + nrm[2] * nrm[2]);
  if (!(nn > 0) || !std::isfinite(nn)) throw Error(MGM_E_NONFINITE, "zero or non-finite normal");
  double n[3] = {nrm[0] / nn, nrm[1] / nn, nrm[2] / nn};
  int ax = 0;
  for (int a = 1; a < 3; ++a)
    if (std::fabs(n[a]) < std::fabs(n[ax])) ax = a;
  double e[3] = {0, 0, 0};
  e[ax] = 1.0;
  for (int a = 0; a < 3; ++a) t1[a] = e[a] - n[ax] * n[a];
  double l = std::sqrt((t1[0] * t1[0] + t1[1] * t1[1]) + t1[2] * t1[2]);
  for (int a = 0; a < 3; ++a) t1[a] /= l;
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

}  // namespace

void project_stencil(const double* xyz, const double* nrm, int64_t i, const int32_t* st, int ns, double* xh) {
  double t1[3], t2[3];
  tangent_basis(nrm + 3 * i, t1, t2);
  for (int j = 0; j < ns; ++j) {
    const double* xj = xyz + 3 * int64_t(st[j]);
    double d[3] = {xj[0] - xyz[3 * i], xj[1] - xyz[3 * i + 1], xj[2] - xyz[3 * i + 2]};
    xh[2 * j] = (t1[0] * d[0] + t1[1] * d[1]) + t1[2] * d[2];
    xh[2 * j + 1] = (t2[0] * d[0] + t2[1] * d[1]) + t2[2] * d[2];
  }
}

namespace {

inline double ipow(double x, int e) {
  double r = 1.0;
  for (int t = 0; t < e; ++t) r *= x;
  return r;
}

// monomial exponents ordered by total degree, then descending power of x
void monomials(int deg, std::vector<int>& ea, std::vector<int>& eb) {
  ea.clear();
  eb.clear();
  for (int d = 0; d <= deg; ++d)
    for (int b = 0; b <= d; ++b) {
      ea.push_back(d - b);
      eb.push_back(b);
    }
}

}  // namespace

void stencil_weights_host(const double* xyz, const double* nrm, int64_t n, const int32_t* sten, int ns,
                          const mgm_params& p, std::vector<double>& w) {
  const int deg = p.poly_degree;
  std::vector<int> ea, eb;
  monomials(deg, ea, eb);
  const int L = int(ea.size());
  w.assign(size_t(n) * ns, 0.0);
  if (p.disc == MGM_RBFFD) {
    const int m = 2 * p.phs_order + 1;
    const int sz = ns + L;
    parallel_for(n, [&](int64_t b, int64_t e) {
      std::vector<double> xh(2 * ns), M(size_t(sz) * sz), rhs(sz);
      std::vector<int> piv(sz);
      for (int64_t i = b; i < e; ++i) {
        const int32_t* st = sten + i * ns;
        project_stencil(xyz, nrm, i, st, ns, xh.data());
        double s = 0.0;
        for (int j = 0; j < ns; ++j)
          s = std::max(s, std::sqrt(xh[2 * j] * xh[2 * j] + xh[2 * j + 1] * xh[2 * j + 1]));
        for (int j = 0; j < 2 * ns; ++j) xh[j] /= s;
        std::fill(M.begin(), M.end(), 0.0);
        for (int j = 0; j < ns; ++j) {
          for (int k = 0; k < ns; ++k) {
            double dx = xh[2 * j] - xh[2 * k], dy = xh[2 * j + 1] - xh[2 * k + 1];
            M[size_t(j) * sz + k] = ipow(std::sqrt(dx * dx + dy * dy), m);
          }
          for (int q = 0; q < L; ++q) {
            double v = ipow(xh[2 * j], ea[q]) * ipow(xh[2 * j + 1], eb[q]);
            M[size_t(j) * sz + ns + q] = v;
            M[size_t(ns + q) * sz + j] = v;
          }
          double r = std::sqrt(xh[2 * j] * xh[2 * j] + xh[2 * j + 1] * xh[2 * j + 1]);
          rhs[j] = double(m) * double(m) * ipow(r, m - 2);
        }
        for (int q = 0; q < L; ++q)
          rhs[ns + q] = ((ea[q] == 2 && eb[q] == 0) || (ea[q] == 0 && eb[q] == 2)) ? 2.0 : 0.0;
        if (!lu_factor(M.data(), sz, piv.data()))
          throw Error(MGM_E_STENCIL_SINGULAR, "RBF-FD stencil system singular at node " + std::to_string(i));
        lu_solve(M.data(), sz, piv.data(), rhs.data());
        const double s2 = s * s;
        for (int j = 0; j < ns; ++j) w[size_t(i) * ns + j] = rhs[j] / s2;
      }
    });
  } else {
    // pass 1: stencil radii rho_i in each node's own tangent plane
    std::vector<double> rho(n);
    parallel_for(n, [&](int64_t b, int64_t e) {
      std::vector<double> xh(2 * ns);
      for (int64_t i = b; i < e; ++i) {
        project_stencil(xyz, nrm, i, sten + i * ns, ns, xh.data());
        double r2 = 0.0;
        for (int j = 0; j < ns; ++j) r2 = std::max(r2, xh[2 * j] * xh[2 * j] + xh[2 * j + 1] * xh[2 * j + 1]);
        rho[i] = std::sqrt(r2);
      }
    });
    const double alpha = p.gfd_alpha;
    parallel_for(n, [&](int64_t b, int64_t e) {
      std::vector<double> xh(2 * ns), B(size_t(ns) * L), sw(ns), v(ns), y(ns), z(L), lp(L), rdiag(L);
      for (int64_t i = b; i < e; ++i) {
        const int32_t* st = sten + i * ns;
        project_stencil(xyz, nrm, i, st, ns, xh.data());
        const double s = rho[i];
        for (int j = 0; j < ns; ++j) {
          double r2 = xh[2 * j] * xh[2 * j] + xh[2 * j + 1] * xh[2 * j + 1];
          double rj = rho[st[j]];
          sw[j] = std::sqrt(std::exp(-alpha * r2 / (s * s + rj * rj)));
        }
        for (int j = 0; j < 2 * ns; ++j) xh[j] /= s;
        for (int j = 0; j < ns; ++j)
          for (int q = 0; q < L; ++q)
            B[size_t(j) * L + q] = sw[j] * ipow(xh[2 * j], ea[q]) * ipow(xh[2 * j + 1], eb[q]);
        // Householder QR, reflectors stored below the diagonal (v_k[k] kept in v0[k])
        std::vector<double> v0(L), beta(L);
        for (int k = 0; k < L; ++k) {
          double nx = 0.0;
          for (int j = k; j < ns; ++j) nx += B[size_t(j) * L + k] * B[size_t(j) * L + k];
          nx = std::sqrt(nx);
          double x0 = B[size_t(k) * L + k];
          double a = (x0 >= 0) ? -nx : nx;
          double vk = x0 - a;
          double bt = vk * vk;
          for (int j = k + 1; j < ns; ++j) bt += B[size_t(j) * L + k] * B[size_t(j) * L + k];
          v0[k] = vk;
          beta[k] = bt;
          rdiag[k] = a;
          if (bt == 0.0) continue;
          for (int q = k + 1; q < L; ++q) {
            double d = vk * B[size_t(k) * L + q];
            for (int j = k + 1; j < ns; ++j) d += B[size_t(j) * L + k] * B[size_t(j) * L + q];
            double f = 2.0 * d / bt;
            B[size_t(k) * L + q] -= f * vk;
            for (int j = k + 1; j < ns; ++j) B[size_t(j) * L + q] -= f * B[size_t(j) * L + k];
          }
        }
        if (!(std::fabs(rdiag[L - 1]) > 1e-13 * std::fabs(rdiag[0])))
          throw Error(MGM_E_STENCIL_SINGULAR, "GFD stencil not unisolvent at node " + std::to_string(i));
        for (int q = 0; q < L; ++q)
          lp[q] = ((ea[q] == 2 && eb[q] == 0) || (ea[q] == 0 && eb[q] == 2)) ? 2.0 : 0.0;
        // R^T z = lp (forward substitution), R upper with diagonal rdiag
        for (int q = 0; q < L; ++q) {
          double t = lp[q];
          for (int r = 0; r < q; ++r) t -= B[size_t(r) * L + q] * z[r];
          z[q] = t / rdiag[q];
        }
        // y = Q [z; 0] = H_0 H_1 ... H_{L-1} [z; 0]
        std::fill(y.begin(), y.end(), 0.0);
        for (int q = 0; q < L; ++q) y[q] = z[q];
        for (int k = L - 1; k >= 0; --k) {
          if (beta[k] == 0.0) continue;
          double d = v0[k] * y[k];
          for (int j = k + 1; j < ns; ++j) d += B[size_t(j) * L + k] * y[j];
          double f = 2.0 * d / beta[k];
          y[k] -= f * v0[k];
          for (int j = k + 1; j < ns; ++j) y[j] -= f * B[size_t(j) * L + k];
        }
        const double s2 = s * s;
        for (int j = 0; j < ns; ++j) w[size_t(i) * ns + j] = sw[j] * y[j] / s2;
      }
    });
  }
}

// Tangent-plane RBF-FD surface gradient (Sec. 6.3 applies it in the heat
// method; the construction is that of Sec. 2.2 with first derivatives): the
// PHS r^m + degree-deg saddle system of the stencil, solved for the
// right-hand sides d/dxh and d/dyh of the basis at the centre
// (d/dx |x - x_j|^m at 0 = -m |x_j|^(m-2) x_j, and 1 for the monomial x),
// then W_ij = (g1_ij t1_i + g2_ij t2_i) / s_i, three doubles per entry.
void surface_gradient_weights_host(const double* xyz, const double* nrm, int64_t n, const int32_t* sten, int ns,
                                   int phs_order, int deg, std::vector<double>& W) {
  if (phs_order < 1) throw Error(MGM_E_ARG, "gradient weights need phs_order >= 1");
  std::vector<int> ea, eb;
  monomials(deg, ea, eb);
  const int L = int(ea.size());
  if (ns < L) throw Error(MGM_E_ARG, "gradient stencil smaller than the polynomial space");
  const int m = 2 * phs_order + 1;
  const int sz = ns + L;
  W.assign(size_t(n) * ns * 3, 0.0);
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<double> xh(2 * ns), M(size_t(sz) * sz), r1(sz), r2(sz);
    std::vector<int> piv(sz);
    for (int64_t i = b; i < e; ++i) {
      const int32_t* st = sten + i * ns;
      project_stencil(xyz, nrm, i, st, ns, xh.data());
      double s = 0.0;
      for (int j = 0; j < ns; ++j) s = std::max(s, std::sqrt(xh[2 * j] * xh[2 * j] + xh[2 * j + 1] * xh[2 * j + 1]));
      for (int j = 0; j < 2 * ns; ++j) xh[j] /= s;
      std::fill(M.begin(), M.end(), 0.0);
      for (int j = 0; j < ns; ++j) {
        for (int k = 0; k < ns; ++k) {
          double dx = xh[2 * j] - xh[2 * k], dy = xh[2 * j + 1] - xh[2 * k + 1];
          M[size_t(j) * sz + k] = ipow(std::sqrt(dx * dx + dy * dy), m);
        }
        for (int q = 0; q < L; ++q) {
          double v = ipow(xh[2 * j], ea[q]) * ipow(xh[2 * j + 1], eb[q]);
          M[size_t(j) * sz + ns + q] = v;
          M[size_t(ns + q) * sz + j] = v;
        }
        double r = std::sqrt(xh[2 * j] * xh[2 * j] + xh[2 * j + 1] * xh[2 * j + 1]);
        double c = -double(m) * ipow(r, m - 2);
        r1[j] = c * xh[2 * j];
        r2[j] = c * xh[2 * j + 1];
      }
      for (int q = 0; q < L; ++q) {
        r1[ns + q] = (ea[q] == 1 && eb[q] == 0) ? 1.0 : 0.0;
        r2[ns + q] = (ea[q] == 0 && eb[q] == 1) ? 1.0 : 0.0;
      }
      if (!lu_factor(M.data(), sz, piv.data()))
        throw Error(MGM_E_STENCIL_SINGULAR, "gradient stencil system singular at node " + std::to_string(i));
      lu_solve(M.data(), sz, piv.data(), r1.data());
      lu_solve(M.data(), sz, piv.data(), r2.data());
      double t1[3], t2[3];
      tangent_basis(nrm + 3 * i, t1, t2);
      for (int j = 0; j < ns; ++j)
        for (int a = 0; a < 3; ++a) W[(size_t(i) * ns + j) * 3 + a] = (r1[j] * t1[a] + r2[j] * t2[a]) / s;
    }
  });
}

}  // namespace mgm
