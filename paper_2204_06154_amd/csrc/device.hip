// Device hierarchy, V-cycle orchestration, Krylov solvers and the C ABI.
//
// Layout in HBM. Every smoothed level j is stored in a permuted row order:
// rows grouped by smoother colour (colour 0 first), and within a colour by a
// 3-D Morton key of the points, so each colour phase streams one contiguous
// row range and its gathers stay spatially local. Row-major CSR (fixed width
// on the fine level), int32 column indices in the permuted numbering, values
// in FP64 and, built on demand, FP32 or FP16 with one FP32 scale per row.
// P_j is a fixed-width (m) row-major table, R_j = P_j^T is CSR, both in
// permuted numbering; the coarsest level keeps its natural order and a dense
// FP64 inverse of its (bordered) operator.
//
// The V-cycle (Alg. 3, zero initial guess, bordered reading of Sec. 4.4) is
// one stream-ordered sequence of kernels on fixed internal buffers and is
// captured once per precision as a HIP graph; callers copy their vector in
// (permute + cast) and out around the graph launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <utility>

#include "ctx.h"
#include "kernels_learned.h"
#include "patch_ops.h"

namespace mgm {

thread_local std::string g_last_error;

static uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
  };
  return spread(x) | spread(y) << 1 | spread(z) << 2;
}

static int choose_G(double mean_len) {
  if (mean_len <= 6) return 2;
  if (mean_len <= 14) return 4;
  if (mean_len <= 40) return 8;
  return 16;
}

// Build the device form of every level (FP64 values).
static void upload(mgm_ctx* c) {
  HostHierarchy& H = c->H;
  const int p = int(H.lv.size());
  c->lv.assign(p, DevLevel());
  std::vector<std::vector<int32_t>> iperm(p);
  // permutations
  for (int j = 0; j < p; ++j) {
    const HostLevel& h = H.lv[j];
    DevLevel& d = c->lv[j];
    d.n = h.n;
    iperm[j].resize(h.n);
    if (j == p - 1) {
      std::iota(iperm[j].begin(), iperm[j].end(), 0);
      continue;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < h.n; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], h.xyz[3 * i + a]);
        hi[a] = std::max(hi[a], h.xyz[3 * i + a]);
      }
    double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    if (!(ext > 0)) ext = 1.0;
    std::vector<uint64_t> key(h.n);
    for (int i = 0; i < h.n; ++i) {
      uint32_t q[3];
      for (int a = 0; a < 3; ++a) q[a] = uint32_t(std::min(2097151.0, std::floor((h.xyz[3 * i + a] - lo[a]) / ext * 2097151.0)));
      key[i] = morton3(q[0], q[1], q[2]);
    }
    std::vector<int32_t> order(h.n);
    std::iota(order.begin(), order.end(), 0);
    d.ncol = h.ncolours;
    if (h.patched) {
      // rows by (patch colour, patch, local colour, Morton rank): patches contiguous
      std::vector<int32_t> mrank(h.n);
      for (int t = 0; t < h.n; ++t) mrank[h.morton[t]] = t;
      std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        int pa = h.pcolour[h.patch[a]], pb = h.pcolour[h.patch[b]];
        if (pa != pb) return pa < pb;
        if (h.patch[a] != h.patch[b]) return h.patch[a] < h.patch[b];
        if (h.lcolour[a] != h.lcolour[b]) return h.lcolour[a] < h.lcolour[b];
        return mrank[a] < mrank[b];
      });
      d.patched = true;
    } else {
      std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (h.colour[a] != h.colour[b]) return h.colour[a] < h.colour[b];
        if (key[a] != key[b]) return key[a] < key[b];
        return a < b;
      });
      d.cstart.assign(h.ncolours + 1, 0);
      for (int i = 0; i < h.n; ++i) d.cstart[h.colour[i] + 1]++;
      for (int k = 0; k < h.ncolours; ++k) d.cstart[k + 1] += d.cstart[k];
    }
    for (int t = 0; t < h.n; ++t) iperm[j][order[t]] = t;
    d.perm = track(c, dupload(order));
  }
  const bool bord = c->p.problem == MGM_POISSON;
  for (int j = 0; j < p; ++j) {
    const HostLevel& h = H.lv[j];
    DevLevel& d = c->lv[j];
    const int n = h.n;
    d.e64 = track(c, dalloc<double>(n + 1));
    d.f64 = track(c, dalloc<double>(n + 1));
    d.res64 = track(c, dalloc<double>(n + 1));
    d.e32 = track(c, dalloc<float>(n + 1));
    d.f32 = track(c, dalloc<float>(n + 1));
    d.res32 = track(c, dalloc<float>(n + 1));
    if (bord) {
      std::vector<double> bp(n);
      for (int i = 0; i < n; ++i) bp[iperm[j][i]] = h.b[i];
      d.b64 = track(c, dupload(bp));
      std::vector<float> bf(bp.begin(), bp.end());
      d.b32 = track(c, dupload(bf));
    }
    if (j == p - 1) continue;
    // permuted CSR of L_j
    std::vector<int32_t> order(n);
    for (int i = 0; i < n; ++i) order[iperm[j][i]] = i;
    std::vector<int32_t> rp(n + 1, 0), cl;
    std::vector<double> vl, diag(n, 0.0);
    cl.reserve(h.L.nnz());
    vl.reserve(h.L.nnz());
    bool fixed = true;
    int w0 = h.L.ptr[1] - h.L.ptr[0];
    for (int pos = 0; pos < n; ++pos) {
      int i = order[pos];
      int len = h.L.ptr[i + 1] - h.L.ptr[i];
      if (len != w0) fixed = false;
      for (int k = h.L.ptr[i]; k < h.L.ptr[i + 1]; ++k) {
        cl.push_back(iperm[j][h.L.col[k]]);
        vl.push_back(h.L.val[k]);
        if (h.L.col[k] == i) diag[pos] = h.L.val[k];
      }
      rp[pos + 1] = int32_t(cl.size());
    }
    d.nnz = int64_t(cl.size());
    d.W = fixed ? w0 : 0;
    d.rowlen_prefix.assign(rp.begin(), rp.end());
    d.G = choose_G(double(d.nnz) / n);
    d.rowptr = track(c, dupload(rp));
    d.col = track(c, dupload(cl));
    d.v64 = track(c, dupload(vl));
    std::vector<double> dinv(n);
    for (int i = 0; i < n; ++i) dinv[i] = 1.0 / diag[i];
    d.dinv64 = track(c, dupload(dinv));
    if (d.patched) {
      // slots = patches in permuted order. ELL per slot with the level's
      // width w (a multiple of kPatchG) and a fixed stride of block rows, so
      // an entry's address follows from (slot, entry, row) alone.
      const int block = c->p.gs_block;
      if (block < 1 || block > kPatch) throw Error(MGM_E_ARG, "gs_block exceeds the patch kernels' rows per workgroup");
      std::vector<int32_t> ps, pn, lc(n), pci;
      std::vector<double> pv;
      std::vector<int32_t> prow;
      int maxw = 0;
      for (int r = 0; r < n; ++r) maxw = std::max(maxw, rp[r + 1] - rp[r]);
      const int w = (maxw + kPatchG - 1) / kPatchG * kPatchG;
      d.pw = w / kPatchG;
      d.pblock = block;
      d.pc_start.assign(1, 0);
      int prev_pc = -1;
      for (int pos = 0; pos < n;) {
        const int i0 = order[pos];
        const int patch = h.patch[i0];
        const int pcol = h.pcolour[patch];
        while (prev_pc < pcol) {
          if (prev_pc >= 0) d.pc_start.push_back(int(ps.size()));
          ++prev_pc;
        }
        int end = pos;
        while (end < n && h.patch[order[end]] == patch) ++end;
        const int nr = end - pos;
        if (nr > block) throw Error(MGM_E_ARG, "patch larger than the block size");
        int ncl = 0;
        for (int t = 0; t < nr; ++t) ncl = std::max(ncl, h.lcolour[order[pos + t]] + 1);
        ps.push_back(pos);
        pn.push_back(ncl);
        const size_t base = pv.size();
        pv.resize(base + size_t(w) * block, 0.0);
        pci.resize(base + size_t(w) * block, pos);   // padding entries: value 0, a valid column
        prow.resize(base + size_t(w) * block, pos);
        for (int t = 0; t < nr; ++t) {
          const int r = pos + t;
          const int len = rp[r + 1] - rp[r];
          for (int k = 0; k < w; ++k) {
            const size_t e = base + (size_t(k / kPatchG) * block + t) * kPatchG + (k % kPatchG);
            prow[e] = r;
            if (k < len) {
              pv[e] = vl[rp[r] + k];
              pci[e] = cl[rp[r] + k];
            } else {
              pci[e] = r;
            }
          }
        }
        pos = end;
      }
      while (prev_pc < h.npcolours) {
        d.pc_start.push_back(int(ps.size()));
        ++prev_pc;
      }
      d.pc_start.resize(h.npcolours + 1);
      ps.push_back(n);
      for (int pos = 0; pos < n; ++pos) lc[pos] = h.lcolour[order[pos]];
      // width class of the patch kernels: entries per row rounded up to a
      // multiple of 8 (24 .. 96), so a row carries few padding entries
      d.wmax = std::max(24, (maxw + 7) / 8 * 8);
      d.pc_nnz.assign(h.npcolours, 0);
      d.pc_rows.assign(h.npcolours, 0);
      for (int pc = 0; pc < h.npcolours; ++pc)
        for (int s = d.pc_start[pc]; s < d.pc_start[pc + 1]; ++s) {
          d.pc_nnz[pc] += int64_t(rp[ps[s + 1]] - rp[ps[s]]);
          d.pc_rows[pc] += ps[s + 1] - ps[s];
        }
      d.pstart_host_slots = int(ps.size()) - 1;
      {
        // one-launch sweeps: the coupled slots of every slot (both directions:
        // a slot that reads another must also be waited for by it) and the
        // row range of each slot's patch colour
        const int nsl = d.pstart_host_slots;
        std::vector<int32_t> slot_of(n), scol(nsl);
        for (int sl = 0; sl < nsl; ++sl)
          for (int r = ps[sl]; r < ps[sl + 1]; ++r) slot_of[r] = sl;
        for (int pc = 0; pc < h.npcolours; ++pc)
          for (int sl = d.pc_start[pc]; sl < d.pc_start[pc + 1]; ++sl) scol[sl] = pc;
        std::vector<std::vector<int32_t>> nbl(nsl);
        for (int sl = 0; sl < nsl; ++sl)
          for (int r = ps[sl]; r < ps[sl + 1]; ++r)
            for (int k = rp[r]; k < rp[r + 1]; ++k) {
              const int q = slot_of[cl[k]];
              if (q != sl) {
                nbl[sl].push_back(q);
                nbl[q].push_back(sl);
              }
            }
        bool ok = true;
        std::vector<int32_t> nbptr(nsl + 1, 0), nb, crow(2 * size_t(nsl));
        for (int sl = 0; sl < nsl; ++sl) {
          auto& v = nbl[sl];
          std::sort(v.begin(), v.end());
          v.erase(std::unique(v.begin(), v.end()), v.end());
          for (int q : v) ok = ok && scol[q] != scol[sl];
          nb.insert(nb.end(), v.begin(), v.end());
          nbptr[sl + 1] = int32_t(nb.size());
          crow[2 * size_t(sl)] = ps[d.pc_start[scol[sl]]];
          crow[2 * size_t(sl) + 1] = ps[d.pc_start[scol[sl] + 1]];
        }
        if (nb.empty()) nb.push_back(0);
        d.flow_ok = ok && nsl > 0;
        d.fl_nbptr = track(c, dupload(nbptr));
        d.fl_nb = track(c, dupload(nb));
        d.fl_crow = track(c, dupload(crow));
        d.fl_ticket = track(c, dalloc<unsigned long long>(1));
        d.fl_flag = track(c, dalloc<unsigned>(nsl));
        HIPCHECK(hipMemset(d.fl_ticket, 0, sizeof(unsigned long long)));
        HIPCHECK(hipMemset(d.fl_flag, 0, sizeof(unsigned) * nsl));
      }
      {
        // staged halo: per slot, the distinct out-of-patch rows its entries
        // reference (ascending), and the columns rewritten to the in-patch
        // row or kPatch + the place in that list
        const int nsl = int(ps.size()) - 1;
        std::vector<int32_t> hstart(nsl + 1, 0), hrows, pch(pci.size());
        std::vector<std::vector<int32_t>> lists(nsl);
        const size_t slot_len = size_t(d.pw) * kPatchG * block;
        parallel_for(nsl, [&](int64_t b, int64_t e1) {  // slots are independent
          for (int64_t sl = b; sl < e1; ++sl) {
            auto& rows = lists[size_t(sl)];
            const size_t e0 = size_t(sl) * slot_len;
            for (size_t e = e0; e < e0 + slot_len; ++e)
              if (pci[e] < ps[sl] || pci[e] >= ps[sl + 1]) rows.push_back(pci[e]);
            std::sort(rows.begin(), rows.end());
            rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
            for (size_t e = e0; e < e0 + slot_len; ++e) {
              const int32_t cc = pci[e];
              pch[e] = (cc >= ps[sl] && cc < ps[sl + 1])
                           ? cc - ps[sl]
                           : kPatch + int32_t(std::lower_bound(rows.begin(), rows.end(), cc) - rows.begin());
            }
          }
        }, 8);
        int hmax = 0;
        for (int sl = 0; sl < nsl; ++sl) {
          hmax = std::max(hmax, int(lists[sl].size()));
          hrows.insert(hrows.end(), lists[sl].begin(), lists[sl].end());
          hstart[sl + 1] = int32_t(hrows.size());
        }
        d.halo_ok = hmax <= kMaxHalo;
        if (d.halo_ok) {
          if (hrows.empty()) hrows.push_back(0);
          d.pcolh = track(c, dupload(pch));
          d.fl_hstart = track(c, dupload(hstart));
          d.fl_hrows = track(c, dupload(hrows));
        }
      }
      d.pstart = track(c, dupload(ps));
      d.pncl = track(c, dupload(pn));
      d.lcol = track(c, dupload(lc));
      d.pcolidx = track(c, dupload(pci));
      d.pv64 = track(c, dupload(pv));
      d.hpv = std::move(pv);
      d.hprow = std::move(prow);
    }
    d.hv = std::move(vl);
    d.hdiag = std::move(diag);
    // interpolation P_j (rows: this level's positions; cols: next level's positions)
    const int m = h.m;
    d.m = m;
    d.nnext = H.lv[j + 1].n;
    std::vector<int32_t> pc(size_t(n) * m);
    std::vector<double> pw(size_t(n) * m);
    for (int pos = 0; pos < n; ++pos) {
      int i = order[pos];
      for (int t = 0; t < m; ++t) {
        pc[size_t(pos) * m + t] = iperm[j + 1][h.pidx[size_t(i) * m + t]];
        pw[size_t(pos) * m + t] = h.pw[size_t(i) * m + t];
      }
    }
    d.pcol = track(c, dupload(pc));
    d.p64 = track(c, dupload(pw));
    std::vector<float> pwf(pw.begin(), pw.end());
    d.p32 = track(c, dupload(pwf));
    // R_j = P_j^T (structural entries only), rows in next-level positions
    Csr Pp;
    Pp.nrows = n;
    Pp.ncols = d.nnext;
    Pp.ptr.assign(n + 1, 0);
    for (int pos = 0; pos < n; ++pos) {
      int i = order[pos];
      int cnt = h.injected[i] ? 1 : m;
      Pp.ptr[pos + 1] = Pp.ptr[pos] + cnt;
      for (int t = 0; t < cnt; ++t) {
        Pp.col.push_back(pc[size_t(pos) * m + t]);
        Pp.val.push_back(pw[size_t(pos) * m + t]);
      }
    }
    Csr Rp = transpose(Pp);
    d.rptr = track(c, dupload(Rp.ptr));
    d.rcol = track(c, dupload(Rp.col));
    d.r64 = track(c, dupload(Rp.val));
    std::vector<float> rf(Rp.val.begin(), Rp.val.end());
    d.r32 = track(c, dupload(rf));
  }
  c->cdim = H.coarse_dim;
  c->cinv = track(c, dupload(H.coarse_inv));
  c->rho = track(c, dalloc<double>(p + 1));
  c->mu = track(c, dalloc<double>(p));  // multiplier correction of every level (mu[0]: the fine one)
  c->lam = track(c, dalloc<double>(1));
  // partial sums: one per block of a plain-level residual (at most 16 lanes a
  // row), or one per half slot of a patch-blocked level's row operators
  int64_t maxblk = 1;
  for (auto& d : c->lv) {
    maxblk = std::max<int64_t>(maxblk, nblk(int64_t(d.n) * 16) + 1);
    if (d.patched) maxblk = std::max<int64_t>(maxblk, 2 * int64_t(d.pstart_host_slots) + 1);
  }
  c->partial_len = maxblk;
  c->partial = track(c, dalloc<double>(maxblk));
  c->flow_err = track(c, dalloc<int>(1));
  HIPCHECK(hipMemset(c->flow_err, 0, sizeof(int)));
  HIPCHECK(hipHostMalloc(reinterpret_cast<void**>(&c->hflow_err), sizeof(int), hipHostMallocDefault));
  *c->hflow_err = 0;
  c->flow_wait_ticks = kFlowWaitTicks;
  HIPCHECK(hipMemset(c->mu, 0, sizeof(double) * p));
  HIPCHECK(hipMemset(c->rho, 0, sizeof(double) * (p + 1)));
}

void build_precision(mgm_ctx* c, int prec) {
  if (c->built[prec]) return;
  for (size_t j = 0; j + 1 < c->lv.size(); ++j) {
    DevLevel& d = c->lv[j];
    const int n = d.n;
    if (prec == MGM_FP32) {
      std::vector<float> v(d.hv.begin(), d.hv.end());
      d.v32 = track(c, dupload(v));
      std::vector<float> di(n);
      for (int i = 0; i < n; ++i) di[i] = float(1.0 / d.hdiag[i]);
      d.dinv32 = track(c, dupload(di));
      if (d.patched) {
        std::vector<float> pv(d.hpv.begin(), d.hpv.end());
        d.pv32 = track(c, dupload(pv));
      }
    } else {
      std::vector<int32_t> rp(n + 1);
      HIPCHECK(hipMemcpy(rp.data(), d.rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
      std::vector<float> s(n), di(n);
      std::vector<uint16_t> h(d.hv.size());
      std::vector<int32_t> cl(d.hv.size());
      HIPCHECK(hipMemcpy(cl.data(), d.col, sizeof(int32_t) * cl.size(), hipMemcpyDeviceToHost));
      for (int i = 0; i < n; ++i) {
        double amax = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) amax = std::max(amax, std::fabs(d.hv[k]));
        float sf = float(amax);
        if (sf == 0.0f) sf = 1.0f;
        s[i] = sf;
        double hd = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
          h[k] = f64_to_f16_bits(d.hv[k] / double(sf));
          if (cl[k] == i) {
            _Float16 q;
            std::memcpy(&q, &h[k], 2);
            hd = double(float(q));
          }
        }
        di[i] = float(1.0 / (double(sf) * hd));
      }
      d.s16 = track(c, dupload(s));
      d.dinv16 = track(c, dupload(di));
      if (d.patched) {
        std::vector<uint16_t> ph(d.hpv.size());
        for (size_t e = 0; e < ph.size(); ++e) ph[e] = f64_to_f16_bits(d.hpv[e] / double(s[d.hprow[e]]));
        _Float16* q16 = dalloc<_Float16>(ph.size());
        track(c, q16);
        HIPCHECK(hipMemcpy(q16, ph.data(), ph.size() * 2, hipMemcpyHostToDevice));
        d.pv16 = q16;
      }
      _Float16* p16 = dalloc<_Float16>(h.size());
      track(c, p16);
      HIPCHECK(hipMemcpy(p16, h.data(), h.size() * 2, hipMemcpyHostToDevice));
      d.v16 = p16;
    }
  }
  c->built[prec] = true;
}

// ----------------------------------------------------------- kernel dispatch
template <typename V, typename S, bool SC>
struct Prec;
template <>
struct Prec<double, double, false> {
  static const double* val(const DevLevel& d) { return d.v64; }
  static const double* pval(const DevLevel& d) { return d.pv64; }
  static const double* dinv(const DevLevel& d) { return d.dinv64; }
  static const double* pw(const DevLevel& d) { return d.p64; }
  static const double* rw(const DevLevel& d) { return d.r64; }
  static double* e(DevLevel& d) { return d.e64; }
  static double* f(DevLevel& d) { return d.f64; }
  static double* res(DevLevel& d) { return d.res64; }
  static const double* b(const DevLevel& d) { return d.b64; }
};
template <>
struct Prec<float, float, false> {
  static const float* val(const DevLevel& d) { return d.v32; }
  static const float* pval(const DevLevel& d) { return d.pv32; }
  static const float* dinv(const DevLevel& d) { return d.dinv32; }
  static const float* pw(const DevLevel& d) { return d.p32; }
  static const float* rw(const DevLevel& d) { return d.r32; }
  static float* e(DevLevel& d) { return d.e32; }
  static float* f(DevLevel& d) { return d.f32; }
  static float* res(DevLevel& d) { return d.res32; }
  static const float* b(const DevLevel& d) { return d.b32; }
};
template <>
struct Prec<_Float16, float, true> {
  static const _Float16* val(const DevLevel& d) { return d.v16; }
  static const _Float16* pval(const DevLevel& d) { return d.pv16; }
  static const float* dinv(const DevLevel& d) { return d.dinv16; }
  static const float* pw(const DevLevel& d) { return d.p32; }
  static const float* rw(const DevLevel& d) { return d.r32; }
  static float* e(DevLevel& d) { return d.e32; }
  static float* f(DevLevel& d) { return d.f32; }
  static float* res(DevLevel& d) { return d.res32; }
  static const float* b(const DevLevel& d) { return d.b32; }
};

#define DISPATCH_G(G, ...)                          \
  switch (G) {                                      \
    case 2: { constexpr int GG = 2; __VA_ARGS__; } break;  \
    case 4: { constexpr int GG = 4; __VA_ARGS__; } break;  \
    case 8: { constexpr int GG = 8; __VA_ARGS__; } break;  \
    default: { constexpr int GG = 16; __VA_ARGS__; } break; \
  }

// One patch colour (pc >= 0, one workgroup per patch of that colour) or, with
// pc < 0, the whole sweep in one dataflow launch (one workgroup per patch).
template <typename V, typename S, bool SC>
static void gs_patch_launch(mgm_ctx* c, int j, int pc, bool reverse, bool border, const double* lam, hipStream_t st,
                            bool zero_guess = false) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  const bool flow = pc < 0;
  const int s0 = flow ? 0 : d.pc_start[pc];
  const int ns = flow ? d.pstart_host_slots : d.pc_start[pc + 1] - s0;
  if (ns <= 0) return;
  GsFlow fl{};
  // staged halo: FP64 vectors on every level, 32-bit ones on levels of at
  // most kStageMaxSlots patches
  const bool staged = flow && d.halo_ok && c->p.gs_flow == 1 &&
                      (sizeof(S) == 8 || d.pstart_host_slots <= kStageMaxSlots);
  if (flow)
    fl = GsFlow{d.fl_ticket, d.fl_flag, d.fl_nbptr, d.fl_nb, d.fl_crow, c->flow_err, ns, c->flow_wait_ticks,
                d.fl_hstart, d.fl_hrows};
#define GS_PATCH(WM, BD, FL, HL)                                                                             \
  hipLaunchKernelGGL((k_gs_patch<V, S, WM / kPatchG, SC, BD, FL, HL>), dim3(ns), dim3(kPatch * kPatchG), 0, st, \
                     s0, reverse ? 1 : 0, zero_guess ? 1 : 0, d.pw, d.pblock, d.pstart, d.pncl, d.lcol,       \
                     P::pval(d), HL ? d.pcolh : d.pcolidx, d.s16, P::dinv(d), P::f(d), P::e(d), P::b(d), lam, fl)
#define GS_PATCH_W(WM, FL, HL) \
  if (border) GS_PATCH(WM, true, FL, HL); else GS_PATCH(WM, false, FL, HL);
#define GS_PATCH_F(WM) \
  if (staged) { GS_PATCH_W(WM, true, true) } else if (flow) { GS_PATCH_W(WM, true, false) } else { GS_PATCH_W(WM, false, false) }
  switch (d.wmax) {
    case 24: GS_PATCH_F(24) break;
    case 32: GS_PATCH_F(32) break;
    case 40: GS_PATCH_F(40) break;
    case 48: GS_PATCH_F(48) break;
    case 56: GS_PATCH_F(56) break;
    case 64: GS_PATCH_F(64) break;
    case 72: GS_PATCH_F(72) break;
    case 80: GS_PATCH_F(80) break;
    case 88: GS_PATCH_F(88) break;
    default: GS_PATCH_F(96) break;
  }
#undef GS_PATCH_F
#undef GS_PATCH_W
#undef GS_PATCH
}

// Whole-level residual (MODE kRowResidual) or product (kRowApply) of a
// patched level from its patch ELL: one workgroup per slot.
template <typename V, typename S, bool SC, int MODE, bool BDOT, bool BORDER, typename X = S>
static void rowop_patch_launch(const DevLevel& d, const V* val, const S* f, const X* x, S* out, const S* b,
                               const double* lam, double* partial, hipStream_t st, const S* dinv = nullptr,
                               const S* omega = nullptr, S* xcopy = nullptr) {
  const unsigned ns = unsigned(d.pstart_host_slots);
#define ROWOP(WM)                                                                                           \
  hipLaunchKernelGGL((k_rowop_patch<V, S, X, WM / kPatchG, SC, MODE, BDOT, BORDER>), dim3(2 * ns), dim3(kRowHalf * kPatchG), \
                     0, st, d.pw, d.pblock, d.pstart, val, d.pcolidx, d.s16, f, x, out, b, lam, partial, dinv, omega, \
                     xcopy, d.n)
  switch (d.wmax) {
    case 24: ROWOP(24); break;
    case 32: ROWOP(32); break;
    case 40: ROWOP(40); break;
    case 48: ROWOP(48); break;
    case 56: ROWOP(56); break;
    case 64: ROWOP(64); break;
    case 72: ROWOP(72); break;
    case 80: ROWOP(80); break;
    case 88: ROWOP(88); break;
    default: ROWOP(96); break;
  }
#undef ROWOP
}

template <typename V, typename S, bool SC>
static void gs_sweep(mgm_ctx* c, int j, bool reverse, bool border, const double* lam, hipStream_t st,
                     bool zero_guess = false) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  if (d.patched) {
    if (c->p.gs_flow && d.flow_ok) {
      gs_patch_launch<V, S, SC>(c, j, -1, reverse, border, lam, st, zero_guess);
      return;
    }
    const int npc = int(d.pc_start.size()) - 1;
    for (int t = 0; t < npc; ++t)
      gs_patch_launch<V, S, SC>(c, j, reverse ? npc - 1 - t : t, reverse, border, lam, st, zero_guess);
    return;
  }
  for (int t = 0; t < d.ncol; ++t) {
    int col = reverse ? d.ncol - 1 - t : t;
    int r0 = d.cstart[col], r1 = d.cstart[col + 1];
    if (r1 <= r0) continue;
    unsigned g = nblk(int64_t(r1 - r0) * d.G);
    DISPATCH_G(d.G, if (border) hipLaunchKernelGGL((k_gs_colour<V, S, GG, SC, true>), dim3(g), dim3(kBlock), 0, st, r0, r1, d.W, d.rowptr, d.col,
                       P::val(d), d.s16, P::dinv(d), P::f(d), P::e(d), P::b(d), lam);
               else hipLaunchKernelGGL((k_gs_colour<V, S, GG, SC, false>), dim3(g), dim3(kBlock), 0, st, r0, r1, d.W, d.rowptr, d.col,
                       P::val(d), d.s16, P::dinv(d), P::f(d), P::e(d), P::b(d), lam));
  }
}

// The row operators of level j write one partial sum per block into
// c->partial; its length is fixed at setup from every level's grid.
static void check_partials(const mgm_ctx* c, int64_t blocks) {
  if (blocks > c->partial_len) throw Error(MGM_E_ARG, "row-operator grid exceeds the partial-sum buffer");
}

// res_j = f_j - L_j e_j (bordered: partial sums of b_j . e_j; with_mu: a
// level continuing from an earlier iterate also subtracts b_j mu_j) then
// f_{j+1} = R_j res_j (bordered: rho_{j+1} = rho_j - b_j . e_j).
template <typename V, typename S, bool SC>
static void residual_restrict(mgm_ctx* c, int j, hipStream_t st, bool with_mu = false) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  DevLevel& nx = c->lv[j + 1];
  const bool bord = c->p.problem == MGM_POISSON;
  const double* mu = c->mu + j;
  unsigned g;  // residual blocks = partial sums of b . e
  if (d.patched) {
    g = 2u * unsigned(d.pstart_host_slots);  // one partial per half slot
    check_partials(c, g);
    if (bord && with_mu) rowop_patch_launch<V, S, SC, kRowResidual, true, true>(d, P::pval(d), P::f(d), P::e(d), P::res(d), P::b(d), mu, c->partial, st);
    else if (bord) rowop_patch_launch<V, S, SC, kRowResidual, true, false>(d, P::pval(d), P::f(d), P::e(d), P::res(d), P::b(d), nullptr, c->partial, st);
    else rowop_patch_launch<V, S, SC, kRowResidual, false, false>(d, P::pval(d), P::f(d), P::e(d), P::res(d), P::b(d), nullptr, c->partial, st);
  } else {
    g = nblk(int64_t(d.n) * d.G);
    check_partials(c, g);
    const double* lam = (bord && with_mu) ? mu : nullptr;
    DISPATCH_G(d.G, if (bord) hipLaunchKernelGGL((k_residual<V, S, GG, SC, true>), dim3(g), dim3(kBlock), 0, st, d.n, d.W, d.rowptr, d.col,
                       P::val(d), d.s16, P::f(d), P::e(d), P::res(d), P::b(d), c->partial, lam);
               else hipLaunchKernelGGL((k_residual<V, S, GG, SC, false>), dim3(g), dim3(kBlock), 0, st, d.n, d.W, d.rowptr, d.col,
                       P::val(d), d.s16, P::f(d), P::e(d), P::res(d), P::b(d), c->partial, (const double*)nullptr));
  }
  unsigned gr = nblk(int64_t(nx.n) * kRestrictG);
  if (bord)
    hipLaunchKernelGGL((k_restrict<S, S, true>), dim3(gr), dim3(kBlock), 0, st, nx.n, d.rptr, d.rcol, P::rw(d), P::res(d),
                       P::f(nx), c->partial, int(g), c->rho + j, c->rho + j + 1);
  else
    hipLaunchKernelGGL((k_restrict<S, S, false>), dim3(gr), dim3(kBlock), 0, st, nx.n, d.rptr, d.rcol, P::rw(d), P::res(d),
                       P::f(nx), c->partial, 0, c->rho + j, c->rho + j + 1);
}

// e_j += P_j e_{j+1}; bordered: mu_j = mu_{j+1}, or mu_j += mu_{j+1} when the
// level continues from an earlier iterate (accumulate).
template <typename V, typename S, bool SC>
static void interp_add(mgm_ctx* c, int j, hipStream_t st, bool accumulate = false, S* out = nullptr) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  DevLevel& nx = c->lv[j + 1];
  const bool bord = c->p.problem == MGM_POISSON;
  hipLaunchKernelGGL((k_interp_add<S, S>), dim3(nblk(d.n)), dim3(kBlock), 0, st, d.n, d.m, d.pcol, P::pw(d), P::e(nx), P::e(d),
                     bord ? c->mu + j + 1 : nullptr, bord ? c->mu + j : nullptr, accumulate ? 1 : 0, out);
}

// scratch vector of the learned smoother's ping-pong (sized for the fine level)
template <typename S>
static S* learned_tmp(mgm_ctx* c) {
  return reinterpret_cast<S*>(sizeof(S) == 8 ? static_cast<void*>(c->e_tmp64) : static_cast<void*>(c->e_tmp32));
}

// Learned smoother of level j: s Richardson steps with per-node step weights
// (ping-pong between e and a scratch vector, the result left in e). With
// border (bordered system) the multiplier is held fixed at *lam, as in the
// Gauss-Seidel sweep. from_tmp: the iterate to smooth is in the scratch
// vector (the interpolation wrote it there), not in e.
template <typename V, typename S, bool SC>
static void learned_sweep(mgm_ctx* c, int j, hipStream_t st, bool border, const double* lam, bool zero_start = false,
                          bool from_tmp = false) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  const LearnedLevel& L = c->ls[j];
  S* e = P::e(d);
  S* tmp = learned_tmp<S>(c);
  const S* om = reinterpret_cast<const S*>(sizeof(S) == 8 ? static_cast<const void*>(L.om64)
                                                           : static_cast<const void*>(L.om32));
  const unsigned g = nblk(int64_t(d.n) * d.G);
  auto step = [&](int q, const S* in, S* out) {
    const S* omq = om + size_t(q) * d.n;
    if (d.patched) {
      if (border)
        rowop_patch_launch<V, S, SC, kRowRichardson, false, true>(d, P::pval(d), P::f(d), in, out, P::b(d), lam, nullptr,
                                                                  st, P::dinv(d), omq);
      else
        rowop_patch_launch<V, S, SC, kRowRichardson, false, false>(d, P::pval(d), P::f(d), in, out, nullptr, nullptr,
                                                                   nullptr, st, P::dinv(d), omq);
    } else if (border) {
      DISPATCH_G(d.G, hipLaunchKernelGGL((k_richardson<V, S, GG, SC, true>), dim3(g), dim3(kBlock), 0, st, d.n, d.W,
                                         d.rowptr, d.col, P::val(d), d.s16, P::dinv(d), omq, P::f(d), in, out, P::b(d),
                                         lam));
    } else {
      DISPATCH_G(d.G, hipLaunchKernelGGL((k_richardson<V, S, GG, SC, false>), dim3(g), dim3(kBlock), 0, st, d.n, d.W,
                                         d.rowptr, d.col, P::val(d), d.s16, P::dinv(d), omq, P::f(d), in, out,
                                         (const S*)nullptr, (const double*)nullptr));
    }
  };
  int q = 0;
  S* a = from_tmp ? tmp : e;
  S* b = from_tmp ? e : tmp;
  if (zero_start) {
    // from e = 0 the first step is omega_1 D^-1 f: no operator pass, and it
    // reads no iterate, so it goes to whichever buffer makes the last of the
    // s steps land in e
    S* first = (L.s % 2 == 1) ? e : tmp;
    hipLaunchKernelGGL((k_scale_start<S>), dim3(nblk(d.n)), dim3(kBlock), 0, st, d.n, om, P::dinv(d), P::f(d), first);
    a = first;
    b = first == e ? tmp : e;
    q = 1;
  }
  // the remaining steps ping-pong; if they end in tmp (a start in e with an
  // odd count, or in tmp with an even one) the result is copied back
  for (; q < L.s; ++q) {
    step(q, a, b);
    std::swap(a, b);
  }
  if (a != e) hipLaunchKernelGGL((k_gather<S, S>), dim3(nblk(d.n)), dim3(kBlock), 0, st, d.n, (const int32_t*)nullptr, a, e,
                                 (double*)nullptr);
}

// One visit of level j in a cycle of the given kind (MGM_CYCLE_V/W/F). With
// zero_start the level starts from e_j = 0, mu_j = 0 (Alg. 3); otherwise it
// continues from its current iterate (the second coarse visit of a W or F
// cycle): pre-smoothing uses mu_j, the residual subtracts b_j mu_j and the
// corrections are added to both e_j and mu_j. The coarsest solve is exact,
// so it does not depend on the start.
template <typename V, typename S, bool SC>
static void cycle_enqueue(mgm_ctx* c, int j, int kind, bool zero_start, hipStream_t st) {
  using P = Prec<V, S, SC>;
  const int p = int(c->lv.size());
  const bool bord = c->p.problem == MGM_POISSON;
  if (j == p - 1) {
    DevLevel& cl = c->lv[p - 1];
    hipLaunchKernelGGL((k_coarse_gemv<S>), dim3(nblk(int64_t(c->cdim) * 64)), dim3(kBlock), 0, st, c->cdim, cl.n, c->cinv,
                       P::f(cl), c->rho + (p - 1), P::e(cl), c->mu + (p - 1));
    return;
  }
  DevLevel& d = c->lv[j];
  const double* mu = c->mu + j;
  const bool learned = learned_on(c, j);
  // e_j starts at zero: a patch-blocked first sweep assumes it without reading e_j
  const bool zg = zero_start && (d.patched || learned) && c->p.nu1 > 0;
  if (zero_start && !zg) hipLaunchKernelGGL((k_fill<S>), dim3(nblk(d.n)), dim3(kBlock), 0, st, d.n, P::e(d), S(0));
  for (int s = 0; s < c->p.nu1; ++s) {
    if (learned) learned_sweep<V, S, SC>(c, j, st, bord && !zero_start, mu, zero_start && s == 0);
    else gs_sweep<V, S, SC>(c, j, c->p.pre_smoother == MGM_GS_BWD, bord && !zero_start, mu, st, zg && s == 0);
  }
  residual_restrict<V, S, SC>(c, j, st, !zero_start);
  const int first = kind;
  cycle_enqueue<V, S, SC>(c, j + 1, first, true, st);
  if (kind != MGM_CYCLE_V) cycle_enqueue<V, S, SC>(c, j + 1, kind == MGM_CYCLE_W ? MGM_CYCLE_W : MGM_CYCLE_V, false, st);
  // With an odd number of learned steps per sweep, the interpolation writes
  // e + P e_c into the scratch vector, so that the first post-smoothing sweep
  // ends in e without a copy.
  const bool interp_to_tmp = learned && c->p.nu2 > 0 && c->ls[j].s % 2 == 1;
  S* after = interp_to_tmp ? learned_tmp<S>(c) : P::e(d);
  interp_add<V, S, SC>(c, j, st, !zero_start, interp_to_tmp ? after : nullptr);
  if (j == c->capture_level && c->capture)
    hipLaunchKernelGGL((k_gather<S, double>), dim3(nblk(d.n)), dim3(kBlock), 0, st, d.n, (const int32_t*)nullptr, after,
                       c->capture, (double*)nullptr);
  for (int s = 0; s < c->p.nu2; ++s) {
    if (learned) learned_sweep<V, S, SC>(c, j, st, bord, mu, false, interp_to_tmp && s == 0);
    else gs_sweep<V, S, SC>(c, j, c->p.post_smoother == MGM_GS_BWD, bord, mu, st);
  }
}

template <typename V, typename S, bool SC>
static void vcycle_enqueue(mgm_ctx* c, hipStream_t st) {
  cycle_enqueue<V, S, SC>(c, 0, c->p.cycle, true, st);
}

void flow_check(mgm_ctx* c, hipStream_t st) {
  HIPCHECK(hipMemcpyAsync(c->hflow_err, c->flow_err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (!*c->hflow_err) return;
  // every launch has ended (each wait is bounded): start the numbering of
  // the sweeps afresh on every patch-blocked level
  HIPCHECK(hipMemsetAsync(c->flow_err, 0, sizeof(int), st));
  for (auto& d : c->lv)
    if (d.fl_ticket) {
      HIPCHECK(hipMemsetAsync(d.fl_ticket, 0, sizeof(unsigned long long), st));
      HIPCHECK(hipMemsetAsync(d.fl_flag, 0, sizeof(unsigned) * size_t(d.pstart_host_slots), st));
    }
  HIPCHECK(hipStreamSynchronize(st));
  *c->hflow_err = 0;
  throw Error(MGM_E_SYNC, "a one-launch smoother sweep gave up waiting for a coupled patch; sweeps resynchronised");
}

void invalidate_graphs(mgm_ctx* c) {
  for (int k = 0; k < 3; ++k)
    if (c->graph[k]) {
      (void)hipGraphExecDestroy(c->graph[k]);
      c->graph[k] = nullptr;
    }
}

void vcycle_core(mgm_ctx* c, hipStream_t st) {
  const int prec = c->p.precision;
  build_precision(c, prec);
  if (c->p.use_graph && !c->capture) {
    if (!c->graph[prec]) {
      if (!c->cap) HIPCHECK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
      hipGraph_t g;
      HIPCHECK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
      if (prec == MGM_FP64) vcycle_enqueue<double, double, false>(c, c->cap);
      else if (prec == MGM_FP32) vcycle_enqueue<float, float, false>(c, c->cap);
      else vcycle_enqueue<_Float16, float, true>(c, c->cap);
      HIPCHECK(hipStreamEndCapture(c->cap, &g));
      hipGraphExec_t ex;
      hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHECK(e);
      c->graph[prec] = ex;
    }
    HIPCHECK(hipGraphLaunch(c->graph[prec], st));
  } else {
    if (prec == MGM_FP64) vcycle_enqueue<double, double, false>(c, st);
    else if (prec == MGM_FP32) vcycle_enqueue<float, float, false>(c, st);
    else vcycle_enqueue<_Float16, float, true>(c, st);
    HIPCHECK(hipGetLastError());
  }
}

// z = M v for FP64 vectors in the fine level's permuted order (perm null) or
// in natural order (perm = the fine permutation).
void precond(mgm_ctx* c, const double* v, double* z, const int32_t* perm, hipStream_t st) {
  DevLevel& d = c->lv[0];
  const bool bord = c->p.problem == MGM_POISSON;
  const unsigned g = nblk(d.n);
  if (c->p.precision == MGM_FP64) {
    hipLaunchKernelGGL((k_gather<double, double>), dim3(g), dim3(kBlock), 0, st, d.n, perm, v, d.f64, bord ? c->rho : nullptr);
    vcycle_core(c, st);
    hipLaunchKernelGGL((k_scatter<double, double>), dim3(g), dim3(kBlock), 0, st, d.n, perm, d.e64, z, bord ? c->mu : nullptr);
  } else {
    hipLaunchKernelGGL((k_gather<double, float>), dim3(g), dim3(kBlock), 0, st, d.n, perm, v, d.f32, bord ? c->rho : nullptr);
    vcycle_core(c, st);
    hipLaunchKernelGGL((k_scatter<float, double>), dim3(g), dim3(kBlock), 0, st, d.n, perm, d.e32, z, bord ? c->mu : nullptr);
  }
}

// v = x / |x| (|x|^2 on the device) and the V-cycle's fine-level input cast
// of v in one pass (FGMRES basis vectors are always the next V-cycle input).
static void normalise_to_vcycle(mgm_ctx* c, int64_t n, const double* x, const double* nrm2, double* v, hipStream_t st) {
  DevLevel& d = c->lv[0];
  double* rho = c->p.problem == MGM_POISSON ? c->rho : nullptr;
  if (c->p.precision == MGM_FP64)
    hipLaunchKernelGGL((k_normalise_cast<double>), dim3(nblk(n)), dim3(kBlock), 0, st, int(n), x, nrm2, v, d.f64, d.n, rho);
  else
    hipLaunchKernelGGL((k_normalise_cast<float>), dim3(nblk(n)), dim3(kBlock), 0, st, int(n), x, nrm2, v, d.f32, d.n, rho);
}

// z = widened V-cycle output and y = A z in one pass over the operator
// (patch-blocked fine level); the bordered constraint row y[n] = b . z is left
// as partial sums in c->partial (two per slot) when defer_border, else summed
// by a reduction launch.
static void apply_from_vcycle(mgm_ctx* c, double* z, double* y, hipStream_t st, bool defer_border = false) {
  DevLevel& d = c->lv[0];
  const bool bord = c->p.problem == MGM_POISSON;
  if (bord) check_partials(c, 2 * int64_t(d.pstart_host_slots));
  if (c->p.precision == MGM_FP64) {
    if (bord) rowop_patch_launch<double, double, false, kRowApply, true, true, double>(d, d.pv64, nullptr, d.e64, y, d.b64, c->mu, c->partial, st, nullptr, nullptr, z);
    else rowop_patch_launch<double, double, false, kRowApply, false, false, double>(d, d.pv64, nullptr, d.e64, y, d.b64, c->mu, nullptr, st, nullptr, nullptr, z);
  } else {
    if (bord) rowop_patch_launch<double, double, false, kRowApply, true, true, float>(d, d.pv64, nullptr, d.e32, y, d.b64, c->mu, c->partial, st, nullptr, nullptr, z);
    else rowop_patch_launch<double, double, false, kRowApply, false, false, float>(d, d.pv64, nullptr, d.e32, y, d.b64, c->mu, nullptr, st, nullptr, nullptr, z);
  }
  // constraint row b . z from the operator pass's partial sums (two per slot)
  if (bord && !defer_border)
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, 1, 2 * d.pstart_host_slots, c->partial, y + d.n,
                       (double*)nullptr);
}

// y = A x (FP64 fine operator, permuted order; bordered tail at index n).
void apply_A(mgm_ctx* c, const double* x, double* y, hipStream_t st) {
  DevLevel& d = c->lv[0];
  const bool bord = c->p.problem == MGM_POISSON;
  if (d.patched) {
    if (bord) rowop_patch_launch<double, double, false, kRowApply, false, true>(d, d.pv64, nullptr, x, y, d.b64, x + d.n, nullptr, st);
    else rowop_patch_launch<double, double, false, kRowApply, false, false>(d, d.pv64, nullptr, x, y, d.b64, x + d.n, nullptr, st);
  } else {
    unsigned g = nblk(int64_t(d.n) * d.G);
    DISPATCH_G(d.G, if (bord) hipLaunchKernelGGL((k_spmv<double, double, GG, false, true>), dim3(g), dim3(kBlock), 0, st, d.n, d.W, d.rowptr,
                       d.col, d.v64, nullptr, x, y, d.b64, x + d.n);
               else hipLaunchKernelGGL((k_spmv<double, double, GG, false, false>), dim3(g), dim3(kBlock), 0, st, d.n, d.W, d.rowptr,
                       d.col, d.v64, nullptr, x, y, d.b64, x + d.n));
  }
  if (bord) mdot(c, d.n, d.b64, 0, 1, x, y + d.n, st);  // constraint row b . x
}

// y = A_j x on a level's CSR (FP64, permuted order); bordered: the level's
// bordered operator [L_j b_j; b_j^T 0], the multiplier at index n_j.
void spmv_level64(mgm_ctx* c, int j, const double* x, double* y, hipStream_t st) {
  DevLevel& d = c->lv[j];
  const bool bord = c->p.problem == MGM_POISSON;
  unsigned g = nblk(int64_t(d.n) * d.G);
  DISPATCH_G(d.G, if (bord) hipLaunchKernelGGL((k_spmv<double, double, GG, false, true>), dim3(g), dim3(kBlock), 0, st, d.n,
                                               d.W, d.rowptr, d.col, d.v64, nullptr, x, y, d.b64, x + d.n);
             else hipLaunchKernelGGL((k_spmv<double, double, GG, false, false>), dim3(g), dim3(kBlock), 0, st, d.n, d.W,
                                     d.rowptr, d.col, d.v64, nullptr, x, y, nullptr, nullptr));
  if (bord) mdot(c, d.n, d.b64, 0, 1, x, y + d.n, st);  // constraint row b_j . x
}

template <typename V, typename S, bool SC>
static void precond_level_t(mgm_ctx* c, int j, const double* v, double* z, hipStream_t st) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  const bool bord = c->p.problem == MGM_POISSON;
  const unsigned g = nblk(d.n);
  hipLaunchKernelGGL((k_gather<double, S>), dim3(g), dim3(kBlock), 0, st, d.n, (const int32_t*)nullptr, v, P::f(d),
                     bord ? c->rho + j : nullptr);
  cycle_enqueue<V, S, SC>(c, j, MGM_CYCLE_V, true, st);
  hipLaunchKernelGGL((k_scatter<S, double>), dim3(g), dim3(kBlock), 0, st, d.n, (const int32_t*)nullptr, P::e(d), z,
                     bord ? c->mu + j : nullptr);
}

void precond_level(mgm_ctx* c, int j, const double* v, double* z, hipStream_t st) {
  if (j < 1 || j + 1 >= int(c->lv.size())) throw Error(MGM_E_ARG, "sub-cycle level out of range");
  const int prec = c->p.precision;
  build_precision(c, prec);
  if (prec == MGM_FP64) precond_level_t<double, double, false>(c, j, v, z, st);
  else if (prec == MGM_FP32) precond_level_t<float, float, false>(c, j, v, z, st);
  else precond_level_t<_Float16, float, true>(c, j, v, z, st);
  HIPCHECK(hipGetLastError());
}

// ------------------------------------------------------------------- solvers
void ensure_ws(mgm_ctx* c, int restart) {
  const int64_t n = c->lv[0].n + 1;
  if (!c->vecs) {
    c->ld = (n + 63) / 64 * 64;
    c->vecs = track(c, dalloc<double>(size_t(c->ld) * 12));
    int64_t kp = std::max<int64_t>(int64_t(kRedBlocks) * 202, nblk(n) + 1);
    c->kpart = track(c, dalloc<double>(kp));
    c->dh = track(c, dalloc<double>(1024));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void**>(&c->hpin), 1024 * sizeof(double), hipHostMallocDefault));
    HIPCHECK(hipEventCreateWithFlags(&c->step_done, hipEventDisableTiming));
  }
  if (restart > c->ws_restart) {
    c->V = track(c, dalloc<double>(size_t(c->ld) * (restart + 1)));
    c->Z = track(c, dalloc<double>(size_t(c->ld) * restart));
    c->ws_restart = restart;
  }
}

// out[t] = V[t] . w for t < k (device), deterministic.
void mdot(mgm_ctx* c, int64_t n, const double* V, int64_t ld, int k, const double* w, double* out, hipStream_t st,
          double* host_out) {
  if (k < 1 || k > kMaxDots) throw Error(MGM_E_ARG, "too many simultaneous dot products");
  int nb = int(std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + 2047) / 2048)));
  hipLaunchKernelGGL(k_mdot_partial, dim3(nb, k), dim3(kBlock), 0, st, int(n), V, ld, w, c->kpart);
  hipLaunchKernelGGL(k_reduce_partials, dim3(k), dim3(kBlock), 0, st, k, nb, c->kpart, out, host_out);
}

// Wait for the stream: the host mirrors written by mdot are then current.
void host_wait(hipStream_t st) { HIPCHECK(hipStreamSynchronize(st)); }

void to_host(mgm_ctx* c, const double* d, int k, hipStream_t st) {
  HIPCHECK(hipMemcpyAsync(c->hpin, d, sizeof(double) * k, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
}

// FGMRES queues the next step's preconditioner before reading this step's
// dots unless the last residual reduction, repeated once more, would bring the
// estimate within this factor of the tolerance.
constexpr double kLookaheadMargin = 10.0;

static mgm_status solve_impl(mgm_ctx* c, const double* d_f, double* d_u, const mgm_solve_opts& o, mgm_solve_info& info,
                             double* hist, hipStream_t st) {
  DevLevel& d0 = c->lv[0];
  const bool bord = c->p.problem == MGM_POISSON;
  const int64_t n = d0.n + (bord ? 1 : 0);
  const int m = std::max(1, o.restart);
  ensure_ws(c, o.krylov == MGM_FGMRES ? m : 1);
  const int64_t ld = c->ld;
  double* f = c->vecs;
  double* x = c->vecs + ld;
  double* r = c->vecs + 2 * ld;
  const unsigned g = nblk(n);
  // permute inputs
  hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(d0.n)), dim3(kBlock), 0, st, d0.n, d0.perm, d_f, f, nullptr);
  if (bord) HIPCHECK(hipMemcpyAsync(f + d0.n, d_f + d0.n, sizeof(double), hipMemcpyDeviceToDevice, st));
  if (o.use_x0) {
    hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(d0.n)), dim3(kBlock), 0, st, d0.n, d0.perm, d_u, x, nullptr);
    if (bord) HIPCHECK(hipMemcpyAsync(x + d0.n, d_u + d0.n, sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    hipLaunchKernelGGL((k_fill<double>), dim3(g), dim3(kBlock), 0, st, int(n), x, 0.0);
  }
  mdot(c, n, f, ld, 1, f, c->dh, st, c->hpin);
  host_wait(st);
  const double fnorm = std::sqrt(c->hpin[0]);
  if (!std::isfinite(fnorm)) throw Error(MGM_E_NONFINITE, "non-finite right-hand side");
  info = mgm_solve_info{};
  int hist_n = 0;
  if (hist) hist[hist_n++] = 1.0;
  auto true_res = [&]() {
    apply_A(c, x, r, st);
    hipLaunchKernelGGL(k_rsub, dim3(g), dim3(kBlock), 0, st, int(n), f, r);
    mdot(c, n, r, ld, 1, r, c->dh, st, c->hpin);
    host_wait(st);
    return std::sqrt(c->hpin[0]);
  };
  auto finish = [&](mgm_status s) {
    hipLaunchKernelGGL((k_scatter<double, double>), dim3(nblk(d0.n)), dim3(kBlock), 0, st, d0.n, d0.perm, x, d_u, nullptr);
    if (bord) {
      HIPCHECK(hipMemcpyAsync(d_u + d0.n, x + d0.n, sizeof(double), hipMemcpyDeviceToDevice, st));
      HIPCHECK(hipMemcpyAsync(c->hpin, x + d0.n, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    HIPCHECK(hipStreamSynchronize(st));
    info.lambda = bord ? c->hpin[0] : 0.0;
    flow_check(c, st);
    return s;
  };
  if (fnorm == 0.0) {
    hipLaunchKernelGGL((k_fill<double>), dim3(g), dim3(kBlock), 0, st, int(n), x, 0.0);
    info.rel_res_true = 0.0;
    return finish(MGM_OK);
  }
  const double tol = o.rtol;
  if (o.krylov == MGM_FGMRES) {
    std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
    for (;;) {
      double beta = true_res();
      info.rel_res_true = beta / fnorm;
      if (!std::isfinite(beta)) return finish(MGM_E_NONFINITE);
      if (beta / fnorm <= tol) return finish(MGM_OK);
      if (info.iters >= o.maxit) return finish(MGM_NOT_CONVERGED);
      if (info.iters > 0) info.restarts++;
      double* V = c->V;
      double* Z = c->Z;
      // V0 = r / beta (beta^2 is on device in dh[0]); on a patch-blocked fine
      // level the basis vectors go straight into the V-cycle's input and its
      // output is widened inside the operator pass (no separate casts)
      const bool fused = d0.patched;
      if (fused) normalise_to_vcycle(c, n, r, c->dh, V, st);
      else hipLaunchKernelGGL(k_normalise, dim3(g), dim3(kBlock), 0, st, int(n), r, c->dh, V);
      std::fill(H.begin(), H.end(), 0.0);
      std::fill(gv.begin(), gv.end(), 0.0);
      gv[0] = beta;
      int k = 0;
      // Preconditioner and operator of step j (they need only V_j, which the
      // device writes itself). Step j + 1's are queued before the host waits
      // for step j's dot products, so the device does not idle during the
      // host's Hessenberg update; the stream order, and so every result, is
      // the same. Not done when the residual trend says step j will converge
      // (the queued work would then delay the solution update).
      // The new vector A z_j is built in place in V's column j + 1.
      // Bordered: the new vector's constraint entry stays as partial sums
      // until the first projection's reduction (k_reduce_partials_border).
      const bool defer = fused && bord;
      auto precond_apply = [&](int jj) {
        if (fused) {
          vcycle_core(c, st);
          apply_from_vcycle(c, Z + jj * ld, V + (jj + 1) * ld, st, defer);
        } else {
          precond(c, V + jj * ld, Z + jj * ld, nullptr, st);
          apply_A(c, Z + jj * ld, V + (jj + 1) * ld, st);
        }
      };
      bool queued = false;
      double last_est = beta / fnorm, rate = 1.0;
      for (int j = 0; j < m; ++j) {
        if (!queued) precond_apply(j);
        queued = false;
        info.iters++;
        // CGS2: two projections; the second one's dots include |w|^2 (w is
        // column j + 1), from which the norm of the projected vector follows,
        // and the second update is fused with the normalisation. The dots
        // land on the host directly.
        const double* hp = c->hpin;
        double* wj = V + (j + 1) * ld;
        if (defer) {
          const int64_t ni = d0.n;  // interior rows; the border entry comes from the partial sums
          const int nb = int(std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (ni + 2047) / 2048)));
          hipLaunchKernelGGL(k_mdot_partial, dim3(nb, j + 1), dim3(kBlock), 0, st, int(ni), V, ld, wj, c->kpart);
          hipLaunchKernelGGL(k_reduce_partials_border, dim3(j + 1), dim3(kBlock), 0, st, j + 1, nb, c->kpart, c->dh,
                             c->hpin, c->partial, 2 * d0.pstart_host_slots, V, ld, int(ni), wj);
        } else {
          mdot(c, n, V, ld, j + 1, wj, c->dh, st, c->hpin);
        }
        hipLaunchKernelGGL(k_mupdate, dim3(g), dim3(kBlock), 0, st, int(n), V, ld, j + 1, c->dh, wj);
        mdot(c, n, V, ld, j + 2, wj, c->dh + 256, st, c->hpin + 256);
        if (fused) {
          DevLevel& dl = c->lv[0];
          double* rho = c->p.problem == MGM_POISSON ? c->rho : nullptr;
          if (c->p.precision == MGM_FP64)
            hipLaunchKernelGGL((k_mupdate_normalise<double>), dim3(g), dim3(kBlock), 0, st, int(n), V, ld, j + 1,
                               c->dh + 256, wj, dl.f64, dl.n, rho);
          else
            hipLaunchKernelGGL((k_mupdate_normalise<float>), dim3(g), dim3(kBlock), 0, st, int(n), V, ld, j + 1,
                               c->dh + 256, wj, dl.f32, dl.n, rho);
        } else {
          hipLaunchKernelGGL((k_mupdate_normalise<double>), dim3(g), dim3(kBlock), 0, st, int(n), V, ld, j + 1,
                             c->dh + 256, wj, (double*)nullptr, 0, (double*)nullptr);
        }
        if (j + 1 < m && info.iters < o.maxit && last_est * rate > kLookaheadMargin * tol) {
          HIPCHECK(hipEventRecord(c->step_done, st));
          precond_apply(j + 1);
          queued = true;
          HIPCHECK(hipEventSynchronize(c->step_done));
        } else {
          host_wait(st);
        }
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) {
          H[size_t(i) * m + j] = hp[i] + hp[256 + i];
          hh += hp[256 + i] * hp[256 + i];
        }
        const double hn2 = hp[256 + j + 1] - hh;
        const double hn = hn2 > 0.0 ? std::sqrt(hn2) : (std::isfinite(hn2) ? 0.0 : hn2);
        if (!std::isfinite(hn)) return finish(MGM_E_NONFINITE);
        H[size_t(j + 1) * m + j] = hn;
        for (int i = 0; i < j; ++i) {
          double t = cs[i] * H[size_t(i) * m + j] + sn[i] * H[size_t(i + 1) * m + j];
          H[size_t(i + 1) * m + j] = -sn[i] * H[size_t(i) * m + j] + cs[i] * H[size_t(i + 1) * m + j];
          H[size_t(i) * m + j] = t;
        }
        double den = std::hypot(H[size_t(j) * m + j], H[size_t(j + 1) * m + j]);
        if (den == 0.0) return finish(MGM_E_BREAKDOWN);
        cs[j] = H[size_t(j) * m + j] / den;
        sn[j] = H[size_t(j + 1) * m + j] / den;
        H[size_t(j) * m + j] = den;
        H[size_t(j + 1) * m + j] = 0.0;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        k = j + 1;
        const double est = std::fabs(gv[j + 1]) / fnorm;
        info.rel_res_est = est;
        if (hist && hist_n <= o.maxit) hist[hist_n++] = est;
        rate = last_est > 0.0 ? est / last_est : 1.0;
        last_est = est;
        if (est <= tol || info.iters >= o.maxit || hn == 0.0) break;
      }
      for (int i = k - 1; i >= 0; --i) {
        double s = gv[i];
        for (int t = i + 1; t < k; ++t) s -= H[size_t(i) * m + t] * y[t];
        y[i] = s / H[size_t(i) * m + i];
      }
      HIPCHECK(hipMemcpyAsync(c->dh + 768, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_madd, dim3(g), dim3(kBlock), 0, st, int(n), Z, ld, k, c->dh + 768, x);
    }
  } else if (o.krylov == MGM_BICGSTAB) {
    // vecs layout: f x r w | rhat p v phat | s t shat
    double* rhat = c->vecs + 4 * ld;
    double* p = c->vecs + 5 * ld;
    double* v = c->vecs + 6 * ld;
    double* phat = c->vecs + 7 * ld;
    double* s = c->vecs + 8 * ld;
    double* t = c->vecs + 9 * ld;
    double* shat = c->vecs + 10 * ld;
    for (;;) {
      double rn = true_res();
      info.rel_res_true = rn / fnorm;
      if (!std::isfinite(rn)) return finish(MGM_E_NONFINITE);
      if (rn / fnorm <= tol) return finish(MGM_OK);
      if (info.iters >= o.maxit) return finish(MGM_NOT_CONVERGED);
      if (info.iters > 0) info.restarts++;
      HIPCHECK(hipMemcpyAsync(rhat, r, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      // The step scalars stay on the device (k_bicg_*); the host waits twice
      // per step, for |s| and for |r|, and sees rho and omega there.
      double* sc = c->dh + 640;   // [parity][rho, rv, st, tt] (8 doubles per parity)
      double* hsc = c->hpin + 640;
      for (int k = 0; info.iters < o.maxit; ++k) {
        const int q = k & 1;
        mdot(c, n, rhat, ld, 1, r, sc + q * 8 + kBicgRho, st, hsc + q * 8 + kBicgRho);  // rho = rhat . r
        if (k == 0) HIPCHECK(hipMemcpyAsync(p, r, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        else hipLaunchKernelGGL(k_bicg_p, dim3(g), dim3(kBlock), 0, st, int(n), r, v, p, sc, q);
        precond(c, p, phat, nullptr, st);
        apply_A(c, phat, v, st);
        mdot(c, n, rhat, ld, 1, v, sc + q * 8 + kBicgRv, st, hsc + q * 8 + kBicgRv);      // rhat . v
        hipLaunchKernelGGL(k_bicg_s, dim3(g), dim3(kBlock), 0, st, int(n), r, v, s, sc, q);
        mdot(c, n, s, ld, 1, s, c->dh + 512, st, c->hpin + 512);
        host_wait(st);
        if (hsc[q * 8 + kBicgRho] == 0.0) break;  // the step just queued is discarded
        info.iters++;
        double sn = std::sqrt(c->hpin[512]) / fnorm;
        if (!std::isfinite(sn)) return finish(MGM_E_NONFINITE);
        if (hist && hist_n <= o.maxit) hist[hist_n++] = sn;
        info.rel_res_est = sn;
        if (sn <= tol) {
          hipLaunchKernelGGL(k_bicg_x, dim3(g), dim3(kBlock), 0, st, int(n), phat, (const double*)nullptr,
                             (const double*)nullptr, (const double*)nullptr, x, (double*)nullptr, sc, q);
          break;
        }
        precond(c, s, shat, nullptr, st);
        info.iters++;
        apply_A(c, shat, t, st);
        // [s.t, t.t] (s and t are adjacent); the step's st and tt slots are adjacent too
        mdot(c, n, s, ld, 2, t, sc + q * 8 + kBicgSt, st, hsc + q * 8 + kBicgSt);
        hipLaunchKernelGGL(k_bicg_x, dim3(g), dim3(kBlock), 0, st, int(n), phat, shat, s, t, x, r, sc, q);
        mdot(c, n, r, ld, 1, r, c->dh + 512, st, c->hpin + 512);
        host_wait(st);
        const double omega = hsc[q * 8 + kBicgSt] / hsc[q * 8 + kBicgTt];
        double rn2 = std::sqrt(c->hpin[512]) / fnorm;
        if (hist && hist_n <= o.maxit) hist[hist_n++] = rn2;
        info.rel_res_est = rn2;
        if (rn2 <= tol || omega == 0.0) break;
      }
    }
  } else {  // stationary: u <- u + M (f - A u)
    double* z = c->vecs + 4 * ld;
    for (;;) {
      double rn = true_res();
      info.rel_res_true = rn / fnorm;
      info.rel_res_est = rn / fnorm;
      if (hist && info.iters > 0 && hist_n <= o.maxit) hist[hist_n++] = rn / fnorm;
      if (!std::isfinite(rn)) return finish(MGM_E_NONFINITE);
      if (rn / fnorm <= tol) return finish(MGM_OK);
      if (info.iters >= o.maxit) return finish(MGM_NOT_CONVERGED);
      precond(c, r, z, nullptr, st);
      info.iters++;
      hipLaunchKernelGGL(k_axpby, dim3(g), dim3(kBlock), 0, st, int(n), 1.0, x, 1.0, z, x);
    }
  }
}

// ---------------------------------------------------------------- level ops
template <typename V, typename S, bool SC>
static void level_op_t(mgm_ctx* c, int op, int j, double* x, const double* b, double* y, bool reverse, hipStream_t st) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  const unsigned g = nblk(d.n);
  hipLaunchKernelGGL((k_gather<double, S>), dim3(g), dim3(kBlock), 0, st, d.n, d.perm, x, P::e(d), nullptr);
  if (op == MGM_OP_SMOOTH) {
    hipLaunchKernelGGL((k_gather<double, S>), dim3(g), dim3(kBlock), 0, st, d.n, d.perm, b, P::f(d), nullptr);
    gs_sweep<V, S, SC>(c, j, reverse, c->p.problem == MGM_POISSON, c->lam, st);
    hipLaunchKernelGGL((k_scatter<S, double>), dim3(g), dim3(kBlock), 0, st, d.n, d.perm, P::e(d), x, nullptr);
  } else if (op == MGM_OP_SPMV) {
    if (d.patched) {
      rowop_patch_launch<V, S, SC, kRowApply, false, false>(d, P::pval(d), nullptr, P::e(d), P::res(d), P::b(d), nullptr,
                                                            nullptr, st);
    } else {
      unsigned gg = nblk(int64_t(d.n) * d.G);
      DISPATCH_G(d.G, hipLaunchKernelGGL((k_spmv<V, S, GG, SC, false>), dim3(gg), dim3(kBlock), 0, st, d.n, d.W, d.rowptr,
                                         d.col, P::val(d), d.s16, P::e(d), P::res(d), P::b(d), (const S*)nullptr));
    }
    hipLaunchKernelGGL((k_scatter<S, double>), dim3(g), dim3(kBlock), 0, st, d.n, d.perm, P::res(d), y, nullptr);
  } else if (op == MGM_OP_RESTRICT_RESIDUAL) {
    hipLaunchKernelGGL((k_gather<double, S>), dim3(g), dim3(kBlock), 0, st, d.n, d.perm, b, P::f(d), nullptr);
    residual_restrict<V, S, SC>(c, j, st);
    DevLevel& nx = c->lv[j + 1];
    hipLaunchKernelGGL((k_scatter<S, double>), dim3(nblk(nx.n)), dim3(kBlock), 0, st, nx.n, nx.perm, P::f(nx), y, nullptr);
  } else {
    DevLevel& nx = c->lv[j + 1];
    hipLaunchKernelGGL((k_gather<double, S>), dim3(nblk(nx.n)), dim3(kBlock), 0, st, nx.n, nx.perm, y, P::e(nx), nullptr);
    interp_add<V, S, SC>(c, j, st);
    hipLaunchKernelGGL((k_scatter<S, double>), dim3(g), dim3(kBlock), 0, st, d.n, d.perm, P::e(d), x, nullptr);
  }
  HIPCHECK(hipGetLastError());
}

// Stencil weights by the batched device solver (RBF-FD, S <= 64); host FP64
// path otherwise.
static WeightsFn device_weights_fn(hipStream_t st) {
  return [st](const double* xyz, const double* nrm, int64_t n, const int32_t* sten, int ns, const mgm_params& p,
              std::vector<double>& w) {
    const int L = (p.poly_degree + 1) * (p.poly_degree + 2) / 2;
    if (p.disc != MGM_RBFFD || ns + L > 64) {
      stencil_weights_host(xyz, nrm, n, sten, ns, p, w);
      return;
    }
    double *dx = dalloc<double>(3 * n), *dn = dalloc<double>(3 * n), *dw = dalloc<double>(size_t(n) * ns);
    int32_t* ds = dalloc<int32_t>(size_t(n) * ns);
    int* dst = dalloc<int>(1);
    auto release = [&] {
      (void)hipFree(dx);
      (void)hipFree(dn);
      (void)hipFree(dw);
      (void)hipFree(ds);
      (void)hipFree(dst);
    };
    try {
      HIPCHECK(hipMemcpyAsync(dx, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
      HIPCHECK(hipMemcpyAsync(dn, nrm, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
      HIPCHECK(hipMemcpyAsync(ds, sten, sizeof(int32_t) * n * ns, hipMemcpyHostToDevice, st));
      HIPCHECK(hipMemsetAsync(dst, 0, sizeof(int), st));
      batched_phs_weights_device(dx, dn, ds, n, ns, p.phs_order, p.poly_degree, dw, dst, st);
      w.resize(size_t(n) * ns);
      int status = 0;
      HIPCHECK(hipMemcpyAsync(w.data(), dw, sizeof(double) * n * ns, hipMemcpyDeviceToHost, st));
      HIPCHECK(hipMemcpyAsync(&status, dst, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      if (status) throw Error(MGM_E_STENCIL_SINGULAR, "RBF-FD stencil system singular (device solver)");
    } catch (...) {
      release();
      throw;
    }
    release();
  };
}

void need_device(const mgm_ctx* c) {
  if (c->device < 0) throw Error(MGM_E_ARG, "host-only handle (set up with device -1)");
}

// --------------------------------------------------------------- profiling
// Algorithmic bytes (values + indices of the touched rows, each vector element
// once) of the hot-path kernels, per precision.
static double bval(int prec) { return prec == MGM_FP64 ? 8.0 : (prec == MGM_FP32 ? 4.0 : 2.0); }
static double bvec(int prec) { return prec == MGM_FP64 ? 8.0 : 4.0; }

static double gs_phase_bytes(const mgm_ctx* c, int j, int col, int prec, bool border) {
  const DevLevel& d = c->lv[j];
  const HostLevel& h = c->H.lv[j];
  int64_t rows = d.cstart[col + 1] - d.cstart[col];
  (void)h;
  // nnz of those rows: from the host copy of the permuted values' row lengths
  int64_t nnz = 0;
  if (d.W > 0) nnz = rows * d.W;
  else nnz = d.rowlen_prefix[d.cstart[col + 1]] - d.rowlen_prefix[d.cstart[col]];
  double b = double(nnz) * (bval(prec) + 4.0) + double(rows) * (bvec(prec) /*dinv*/ + 3.0 * bvec(prec));
  if (d.W == 0) b += double(rows + 1) * 4.0;
  if (prec == MGM_FP16) b += 4.0 * double(rows);
  if (border) b += bvec(prec) * double(rows);
  return b;
}

// one patch-colour launch of the patch-blocked smoother
static double gs_patch_bytes(const mgm_ctx* c, int j, int pc, int prec, bool border) {
  const DevLevel& d = c->lv[j];
  const double rows = d.pc_rows[pc];
  double b = double(d.pc_nnz[pc]) * (bval(prec) + 4.0) + rows * (bvec(prec) + 3.0 * bvec(prec) + 4.0);
  if (prec == MGM_FP16) b += 4.0 * rows;
  if (border) b += bvec(prec) * rows;
  return b;
}

static double gs_sweep_bytes(const mgm_ctx* c, int j, int prec, bool border) {
  const DevLevel& d = c->lv[j];
  double b = 0.0;
  if (d.patched) {
    for (int pc = 0; pc + 1 < int(d.pc_start.size()); ++pc) b += gs_patch_bytes(c, j, pc, prec, border);
  } else {
    for (int col = 0; col < d.ncol; ++col) b += gs_phase_bytes(c, j, col, prec, border);
  }
  return b;
}

// one Richardson step of the learned smoother on level j: the operator
// (values + indices), x, f, the output, D^-1 and the step weights once each
// (bordered: b)
static double richardson_bytes(const mgm_ctx* c, int j, int prec, bool border) {
  const DevLevel& d = c->lv[j];
  double b = double(d.nnz) * (bval(prec) + 4.0) + 5.0 * bvec(prec) * d.n;
  if (d.W == 0) b += 4.0 * (d.n + 1);
  if (prec == MGM_FP16) b += 4.0 * d.n;
  if (border) b += bvec(prec) * d.n;
  return b;
}

// one learned sweep: (launches, algorithmic bytes); from zero the first step
// reads omega, D^-1 and f and writes e (no operator pass); from a non-zero
// start in e an odd step count ends with a copy back into e (a start in the
// scratch vector, as after the interpolation, needs none), a launch whose
// bytes are not algorithmic
static std::pair<int, double> learned_sweep_cost(const mgm_ctx* c, int j, int prec, bool border, bool zero_start,
                                                 bool from_tmp = false) {
  const int s = c->ls[j].s;
  if (zero_start) return {s, 4.0 * bvec(prec) * c->lv[j].n + (s - 1) * richardson_bytes(c, j, prec, false)};
  const int copy = (s % 2 == 1) != from_tmp ? 1 : 0;
  return {s + copy, s * richardson_bytes(c, j, prec, border)};
}

static double residual_bytes(const mgm_ctx* c, int j, int prec) {
  const DevLevel& d = c->lv[j];
  double b = double(d.nnz) * (bval(prec) + 4.0) + 3.0 * bvec(prec) * d.n;
  if (d.W == 0) b += 4.0 * (d.n + 1);
  if (prec == MGM_FP16) b += 4.0 * d.n;
  return b;
}

// Algorithmic bytes of one visit of level j (cf. cycle_enqueue), recursively.
static double visit_bytes(const mgm_ctx* c, int prec, int j, int kind, bool zero_start) {
  const int p = int(c->lv.size());
  if (j == p - 1) return 8.0 * double(c->cdim) * c->cdim + bvec(prec) * 2.0 * c->lv[p - 1].n;  // coarse
  const bool bord = c->p.problem == MGM_POISSON;
  const double bt = prec == MGM_FP64 ? 8.0 : 4.0;  // transfer value bytes
  const DevLevel& d = c->lv[j];
  const bool learned = learned_on(c, j);
  double tot = 0.0;
  if (zero_start && !((d.patched || learned) && c->p.nu1 > 0)) tot += bvec(prec) * d.n;  // zero fill
  if (learned) {
    for (int s = 0; s < c->p.nu1; ++s)
      tot += learned_sweep_cost(c, j, prec, bord && !zero_start, zero_start && s == 0).second;
    tot += c->p.nu2 * learned_sweep_cost(c, j, prec, bord, false).second;
  } else {
    tot += c->p.nu1 * gs_sweep_bytes(c, j, prec, bord && !zero_start) + c->p.nu2 * gs_sweep_bytes(c, j, prec, bord);
  }
  tot += residual_bytes(c, j, prec);
  const int64_t nnzR = c->H.lv[j].R.nnz();
  tot += double(nnzR) * (bt + 4.0) + 4.0 * (d.nnext + 1) + bvec(prec) * (d.n + d.nnext);      // restrict
  tot += visit_bytes(c, prec, j + 1, kind, true);
  if (kind != MGM_CYCLE_V) tot += visit_bytes(c, prec, j + 1, kind == MGM_CYCLE_W ? MGM_CYCLE_W : MGM_CYCLE_V, false);
  tot += double(d.n) * d.m * (bt + 4.0) + bvec(prec) * (d.nnext + 2.0 * d.n);                  // interpolate
  return tot;
}

static double vcycle_bytes(const mgm_ctx* c, int prec) { return visit_bytes(c, prec, 0, c->p.cycle, true); }

template <typename V, typename S, bool SC>
static void gs_phase_launch(mgm_ctx* c, int j, int col, hipStream_t st) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  int r0 = d.cstart[col], r1 = d.cstart[col + 1];
  unsigned g = nblk(int64_t(r1 - r0) * d.G);
  DISPATCH_G(d.G, hipLaunchKernelGGL((k_gs_colour<V, S, GG, SC, false>), dim3(g), dim3(kBlock), 0, st, r0, r1, d.W, d.rowptr,
                                     d.col, P::val(d), d.s16, P::dinv(d), P::f(d), P::e(d), P::b(d), c->mu));
}

template <typename V, typename S, bool SC>
static void residual_launch(mgm_ctx* c, int j, hipStream_t st) {
  using P = Prec<V, S, SC>;
  DevLevel& d = c->lv[j];
  if (d.patched) {
    rowop_patch_launch<V, S, SC, kRowResidual, false, false>(d, P::pval(d), P::f(d), P::e(d), P::res(d), P::b(d), nullptr, c->partial, st);
    return;
  }
  unsigned g = nblk(int64_t(d.n) * d.G);
  DISPATCH_G(d.G, hipLaunchKernelGGL((k_residual<V, S, GG, SC, false>), dim3(g), dim3(kBlock), 0, st, d.n, d.W, d.rowptr, d.col,
                                     P::val(d), d.s16, P::f(d), P::e(d), P::res(d), P::b(d), c->partial));
}

static void time_kernel_impl(mgm_ctx* c, int which, int level, int reps, hipStream_t st, double* ms, double* bytes) {
  const int prec = c->p.precision;
  build_precision(c, prec);
  ensure_ws(c, 1);
  const bool all_gs = which == MGM_TK_GS && level == -1;
  if (which < MGM_TK_SPMV || which > MGM_TK_LEARNED) throw Error(MGM_E_ARG, "unknown kernel");
  if (which != MGM_TK_SPMV && which != MGM_TK_VCYCLE && which != MGM_TK_LEARNED && !all_gs &&
      (level < 0 || level + 1 >= int(c->lv.size())))
    throw Error(MGM_E_ARG, "level out of range");
  if (reps < 1) throw Error(MGM_E_ARG, "reps must be >= 1");
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  double total = 0.0, tbytes = 0.0;
  int64_t count = 0;
  auto timed = [&](const std::function<void()>& launch, double b) {
    HIPCHECK(hipEventRecord(e0, st));
    launch();
    HIPCHECK(hipEventRecord(e1, st));
    HIPCHECK(hipEventSynchronize(e1));
    float t = 0.0f;
    HIPCHECK(hipEventElapsedTime(&t, e0, e1));
    total += t;
    tbytes += b;
    ++count;
  };
  DevLevel& d0 = c->lv[0];
  for (int r = 0; r < reps; ++r) {
    if (which == MGM_TK_SPMV) {
      double b = double(d0.nnz) * 12.0 + 16.0 * d0.n + (d0.W == 0 ? 4.0 * (d0.n + 1) : 0.0);
      timed([&] {
        if (d0.patched) {
          rowop_patch_launch<double, double, false, kRowApply, false, false>(d0, d0.pv64, nullptr, c->vecs, c->vecs + c->ld,
                                                                             d0.b64, nullptr, nullptr, st);
          return;
        }
        unsigned g = nblk(int64_t(d0.n) * d0.G);
        DISPATCH_G(d0.G, hipLaunchKernelGGL((k_spmv<double, double, GG, false, false>), dim3(g), dim3(kBlock), 0, st, d0.n, d0.W,
                                            d0.rowptr, d0.col, d0.v64, nullptr, c->vecs, c->vecs + c->ld, d0.b64,
                                            (const double*)nullptr));
      }, b);
    } else if (all_gs) {
      // the smoother launches of one V-cycle, in its order, as one timed batch
      const bool bord = c->p.problem == MGM_POISSON;
      const int p = int(c->lv.size());
      int64_t launches = 0;
      double b = 0.0;
      for (int j = 0; j + 1 < p; ++j) {
        const DevLevel& d = c->lv[j];
        const int per = d.patched ? (c->p.gs_flow && d.flow_ok ? 1 : int(d.pc_start.size()) - 1) : d.ncol;
        launches += int64_t(c->p.nu1 + c->p.nu2) * per;
        b += c->p.nu1 * gs_sweep_bytes(c, j, prec, false) + c->p.nu2 * gs_sweep_bytes(c, j, prec, bord);
      }
      auto sweeps = [&] {
        for (int j = 0; j + 1 < p; ++j) {
          const bool zg = c->lv[j].patched && c->p.nu1 > 0;
          for (int s = 0; s < c->p.nu1; ++s) {
            if (prec == MGM_FP64) gs_sweep<double, double, false>(c, j, c->p.pre_smoother == MGM_GS_BWD, false, c->mu, st, zg && s == 0);
            else if (prec == MGM_FP32) gs_sweep<float, float, false>(c, j, c->p.pre_smoother == MGM_GS_BWD, false, c->mu, st, zg && s == 0);
            else gs_sweep<_Float16, float, true>(c, j, c->p.pre_smoother == MGM_GS_BWD, false, c->mu, st, zg && s == 0);
          }
          for (int s = 0; s < c->p.nu2; ++s) {
            if (prec == MGM_FP64) gs_sweep<double, double, false>(c, j, c->p.post_smoother == MGM_GS_BWD, bord, c->mu, st);
            else if (prec == MGM_FP32) gs_sweep<float, float, false>(c, j, c->p.post_smoother == MGM_GS_BWD, bord, c->mu, st);
            else gs_sweep<_Float16, float, true>(c, j, c->p.post_smoother == MGM_GS_BWD, bord, c->mu, st);
          }
        }
      };
      timed(sweeps, b);
      count += launches - 1;  // timed() counted the batch once
    } else if (which == MGM_TK_LEARNED) {
      // the learned smoother's launches of one V-cycle on every level where it
      // is active, in the cycle's order, as one timed batch
      const bool bord = c->p.problem == MGM_POISSON;
      const int p = int(c->lv.size());
      int64_t launches = 0;
      double b = 0.0;
      for (int j = 0; j + 1 < p; ++j) {
        if (!learned_on(c, j)) continue;
        for (int s = 0; s < c->p.nu1; ++s) {
          const auto cost = learned_sweep_cost(c, j, prec, false, s == 0);
          launches += cost.first;
          b += cost.second;
        }
        for (int s = 0; s < c->p.nu2; ++s) {
          const auto cost = learned_sweep_cost(c, j, prec, bord, false, s == 0 && c->ls[j].s % 2 == 1);
          launches += cost.first;
          b += cost.second;
        }
      }
      if (launches == 0) throw Error(MGM_E_ARG, "no level uses the learned smoother");
      auto sweeps = [&] {
        for (int j = 0; j + 1 < p; ++j) {
          if (!learned_on(c, j)) continue;
          const double* mu = c->mu + j;
          for (int s = 0; s < c->p.nu1; ++s) {
            if (prec == MGM_FP64) learned_sweep<double, double, false>(c, j, st, false, mu, s == 0);
            else if (prec == MGM_FP32) learned_sweep<float, float, false>(c, j, st, false, mu, s == 0);
            else learned_sweep<_Float16, float, true>(c, j, st, false, mu, s == 0);
          }
          for (int s = 0; s < c->p.nu2; ++s) {
            const bool from_tmp = s == 0 && c->ls[j].s % 2 == 1;  // as after the cycle's interpolation
            if (prec == MGM_FP64) learned_sweep<double, double, false>(c, j, st, bord, mu, false, from_tmp);
            else if (prec == MGM_FP32) learned_sweep<float, float, false>(c, j, st, bord, mu, false, from_tmp);
            else learned_sweep<_Float16, float, true>(c, j, st, bord, mu, false, from_tmp);
          }
        }
      };
      timed(sweeps, b);
      count += launches - 1;  // timed() counted the batch once
    } else if (which == MGM_TK_GS && c->lv[level].patched && c->p.gs_flow && c->lv[level].flow_ok) {
      timed([&] {
        if (prec == MGM_FP64) gs_patch_launch<double, double, false>(c, level, -1, false, false, c->mu, st);
        else if (prec == MGM_FP32) gs_patch_launch<float, float, false>(c, level, -1, false, false, c->mu, st);
        else gs_patch_launch<_Float16, float, true>(c, level, -1, false, false, c->mu, st);
      }, gs_sweep_bytes(c, level, prec, false));
    } else if (which == MGM_TK_GS && c->lv[level].patched) {
      DevLevel& d = c->lv[level];
      for (int pc = 0; pc + 1 < int(d.pc_start.size()); ++pc) {
        timed([&] {
          if (prec == MGM_FP64) gs_patch_launch<double, double, false>(c, level, pc, false, false, c->mu, st);
          else if (prec == MGM_FP32) gs_patch_launch<float, float, false>(c, level, pc, false, false, c->mu, st);
          else gs_patch_launch<_Float16, float, true>(c, level, pc, false, false, c->mu, st);
        }, gs_patch_bytes(c, level, pc, prec, false));
      }
    } else if (which == MGM_TK_GS) {
      DevLevel& d = c->lv[level];
      for (int col = 0; col < d.ncol; ++col) {
        if (d.cstart[col + 1] <= d.cstart[col]) continue;
        timed([&] {
          if (prec == MGM_FP64) gs_phase_launch<double, double, false>(c, level, col, st);
          else if (prec == MGM_FP32) gs_phase_launch<float, float, false>(c, level, col, st);
          else gs_phase_launch<_Float16, float, true>(c, level, col, st);
        }, gs_phase_bytes(c, level, col, prec, false));
      }
    } else if (which == MGM_TK_RESIDUAL) {
      timed([&] {
        if (prec == MGM_FP64) residual_launch<double, double, false>(c, level, st);
        else if (prec == MGM_FP32) residual_launch<float, float, false>(c, level, st);
        else residual_launch<_Float16, float, true>(c, level, st);
      }, residual_bytes(c, level, prec));
    } else if (which == MGM_TK_VCYCLE) {
      timed([&] { vcycle_core(c, st); }, vcycle_bytes(c, prec));
    } else {
      throw Error(MGM_E_ARG, "unknown kernel");
    }
  }
  HIPCHECK(hipGetLastError());
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = total / double(count);
  *bytes = tbytes / double(count);
}

mgm_status guard(const std::function<void()>& f) {
  try {
    f();
    return MGM_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return MGM_E_ALLOC;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return MGM_E_ARG;
  }
}

}  // namespace mgm

using namespace mgm;

extern "C" {

void mgm_default_params(mgm_params* p) {
  if (!p) return;
  *p = mgm_params{};
  p->disc = MGM_RBFFD;
  p->phs_order = 3;
  p->poly_degree = 3;
  p->stencil_size = 20;
  p->gfd_alpha = 4.0;
  p->problem = MGM_SCREENED;
  p->mu = 1.0;
  p->interp_size = 3;
  p->coarsen_factor = 4;
  p->n_min = 250;
  p->n_coarse_max = 0;
  p->nu1 = 1;
  p->nu2 = 1;
  p->pre_smoother = MGM_GS_FWD;
  p->post_smoother = MGM_GS_FWD;
  p->precision = MGM_FP64;
  p->use_graph = 1;
  p->device_weights = 1;
  p->device_setup = 1;
  p->gs_block = 256;
  p->gs_max_width = kMaxPatchWidth;
  p->cycle = MGM_CYCLE_V;
  p->gs_flow = 1;
}

mgm_status mgm_setup(const double* h_xyz, const double* h_normals, int64_t n, const mgm_params* params, int32_t device,
                     void* stream, mgm_handle* out) {
  if (!out || !params || !h_xyz || !h_normals) {
    g_last_error = "null argument";
    return MGM_E_ARG;
  }
  *out = nullptr;
  std::unique_ptr<mgm_ctx> c(new mgm_ctx());
  mgm_status s = guard([&] {
    c->device = device;
    c->p = *params;
    if (device < -1) throw Error(MGM_E_ARG, "device must be >= -1");
    if (device >= 0) HIPCHECK(hipSetDevice(device));
    SetupBackend be = host_backend();
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (device >= 0 && params->device_weights) be.weights = device_weights_fn(st);
    if (device >= 0 && params->device_setup) {
      be.knn = [st](const double* q, int64_t nq, const double* d, int64_t nd, int k, std::vector<int32_t>& idx,
                    std::vector<double>& d2) {
        if (k <= 128) knn_device(q, nq, d, nd, k, idx, d2, st);
        else knn_search(q, nq, d, nd, k, idx, d2);
      };
      be.spgemm = [st](const Csr& A, const Csr& B) { return spgemm_device(A, B, st); };
      be.dsatur = [st](const std::vector<int32_t>& lptr, const std::vector<int32_t>& ladj,
                       const std::vector<int32_t>& pstart, std::vector<int32_t>& lc, std::vector<int32_t>& pnlc) {
        dsatur_patches_device(lptr, ladj, pstart, lc, pnlc, st);
      };
    }
    build_hierarchy(h_xyz, h_normals, n, *params, be, c->H);
    if (device >= 0) {
      upload(c.get());
      HIPCHECK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    }
  });
  if (s != MGM_OK) {
    for (void* ptr : c->allocs) (void)hipFree(ptr);
    return s;
  }
  *out = c.release();
  return MGM_OK;
}

mgm_status mgm_set_precision(mgm_handle h, int32_t precision) {
  if (!h || precision < MGM_FP64 || precision > MGM_FP16) {
    g_last_error = "bad handle or precision";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    h->p.precision = precision;
    build_precision(h, precision);
  });
}

mgm_status mgm_vcycle(mgm_handle h, const double* d_r, double* d_z, void* stream) {
  if (!h || !d_r || !d_z || d_r == d_z) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    precond(h, d_r, d_z, h->lv[0].perm, static_cast<hipStream_t>(stream));
    HIPCHECK(hipGetLastError());
  });
}

mgm_status mgm_apply(mgm_handle h, const double* d_x, double* d_y, void* stream) {
  if (!h || !d_x || !d_y || d_x == d_y) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    ensure_ws(h, 1);
    DevLevel& d = h->lv[0];
    const bool bord = h->p.problem == MGM_POISSON;
    double* xp = h->vecs + 2 * h->ld;
    double* yp = h->vecs + 3 * h->ld;
    hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(d.n)), dim3(kBlock), 0, st, d.n, d.perm, d_x, xp, nullptr);
    if (bord) HIPCHECK(hipMemcpyAsync(xp + d.n, d_x + d.n, sizeof(double), hipMemcpyDeviceToDevice, st));
    apply_A(h, xp, yp, st);
    hipLaunchKernelGGL((k_scatter<double, double>), dim3(nblk(d.n)), dim3(kBlock), 0, st, d.n, d.perm, yp, d_y, nullptr);
    if (bord) HIPCHECK(hipMemcpyAsync(d_y + d.n, yp + d.n, sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipGetLastError());
  });
}

mgm_status mgm_solve(mgm_handle h, const double* d_f, double* d_u, const mgm_solve_opts* opts, mgm_solve_info* info,
                     double* h_res_hist, void* stream) {
  if (!h || !d_f || !d_u || !opts || !info || d_f == d_u || opts->restart < 1 || opts->restart > 200 ||
      opts->maxit < 0 || !(opts->rtol >= 0) || opts->krylov < MGM_FGMRES || opts->krylov > MGM_STATIONARY) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  mgm_status res = MGM_OK;
  mgm_status s = guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    res = solve_impl(h, d_f, d_u, *opts, *info, h_res_hist, static_cast<hipStream_t>(stream));
  });
  return s != MGM_OK ? s : res;
}

mgm_status mgm_level_op(mgm_handle h, int32_t op, int32_t level, double* d_x, const double* d_b, double* d_y, double scalar,
                        int32_t reverse, void* stream) {
  if (!h || level < 0 || level + 1 >= int32_t(h->lv.size()) || op < MGM_OP_SMOOTH || op > MGM_OP_INTERP_ADD || !d_x ||
      ((op == MGM_OP_SMOOTH || op == MGM_OP_RESTRICT_RESIDUAL) && !d_b) || (op != MGM_OP_SMOOTH && !d_y)) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    build_precision(h, h->p.precision);
    HIPCHECK(hipMemcpyAsync(h->lam, &scalar, sizeof(double), hipMemcpyHostToDevice, st));
    if (op == MGM_OP_RESTRICT_RESIDUAL && h->p.problem == MGM_POISSON)
      HIPCHECK(hipMemsetAsync(h->rho + level, 0, sizeof(double), st));
    if (h->p.precision == MGM_FP64) level_op_t<double, double, false>(h, op, level, d_x, d_b, d_y, reverse != 0, st);
    else if (h->p.precision == MGM_FP32) level_op_t<float, float, false>(h, op, level, d_x, d_b, d_y, reverse != 0, st);
    else level_op_t<_Float16, float, true>(h, op, level, d_x, d_b, d_y, reverse != 0, st);
    flow_check(h, st);
  });
}

mgm_status mgm_check(mgm_handle h, void* stream) {
  if (!h) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    flow_check(h, static_cast<hipStream_t>(stream));
  });
}

mgm_status mgm_set_flow_wait(mgm_handle h, int64_t ticks) {
  if (!h) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    HIPCHECK(hipDeviceSynchronize());
    h->flow_wait_ticks = ticks < 0 ? kFlowWaitTicks : (unsigned long long)ticks;
    invalidate_graphs(h);  // the bound is a launch argument captured in the graphs
  });
}

mgm_status mgm_time_kernel(mgm_handle h, int32_t which, int32_t level, int32_t reps, void* stream, double* ms,
                           double* bytes) {
  if (!h || !ms || !bytes) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    need_device(h);
    HIPCHECK(hipSetDevice(h->device));
    time_kernel_impl(h, which, level, reps, static_cast<hipStream_t>(stream), ms, bytes);
  });
}

mgm_status mgm_stencils(const double* h_xyz, int64_t n, int32_t k, int32_t* h_idx) {
  if (!h_xyz || !h_idx || n < 1 || k < 1 || k > n) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    std::vector<int32_t> idx;
    std::vector<double> d2;
    knn_search(h_xyz, n, h_xyz, n, k, idx, d2);
    for (int64_t i = 0; i < n; ++i)
      if ((k > 1 && d2[size_t(i) * k + 1] == 0.0) || idx[size_t(i) * k] != i)
        throw Error(MGM_E_DUP_POINTS, "duplicate points in the point cloud");
    std::memcpy(h_idx, idx.data(), idx.size() * sizeof(int32_t));
  });
}

static mgm_status batched_weights_entry(const double* d_xyz, const double* d_normals, int64_t n_points,
                                        const int32_t* d_stencils, int64_t n_systems, int32_t stencil_size,
                                        int32_t phs_order, int32_t poly_degree, double* d_weights, void* stream,
                                        bool mixed) {
  // an empty batch may pass null stencils and weights (it still checks the sizes)
  if (!d_xyz || !d_normals || (n_systems > 0 && (!d_stencils || !d_weights)) || n_points < 1 || n_systems < 0 ||
      stencil_size < 1 || stencil_size > n_points) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  mgm_status res = MGM_OK;
  mgm_status s = guard([&] {
    hipStream_t st = static_cast<hipStream_t>(stream);
    int* dst = dalloc<int>(1);
    int status = 0;
    try {
      HIPCHECK(hipMemsetAsync(dst, 0, sizeof(int), st));
      batched_phs_weights_device(d_xyz, d_normals, d_stencils, n_systems, stencil_size, phs_order, poly_degree,
                                 d_weights, dst, st, mixed);
      HIPCHECK(hipMemcpyAsync(&status, dst, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
    } catch (...) {
      (void)hipFree(dst);
      throw;
    }
    (void)hipFree(dst);
    if (status) {
      g_last_error = "a stencil system is singular";
      res = MGM_E_STENCIL_SINGULAR;
    }
  });
  return s != MGM_OK ? s : res;
}

mgm_status mgm_batched_weights(const double* d_xyz, const double* d_normals, int64_t n_points, const int32_t* d_stencils,
                               int64_t n_systems, int32_t stencil_size, int32_t phs_order, int32_t poly_degree,
                               double* d_weights, void* stream) {
  return batched_weights_entry(d_xyz, d_normals, n_points, d_stencils, n_systems, stencil_size, phs_order, poly_degree,
                               d_weights, stream, false);
}

mgm_status mgm_batched_weights_mixed(const double* d_xyz, const double* d_normals, int64_t n_points,
                                     const int32_t* d_stencils, int64_t n_systems, int32_t stencil_size,
                                     int32_t phs_order, int32_t poly_degree, double* d_weights, void* stream) {
  return batched_weights_entry(d_xyz, d_normals, n_points, d_stencils, n_systems, stencil_size, phs_order, poly_degree,
                               d_weights, stream, true);
}

mgm_status mgm_export(mgm_handle h, int32_t what, int32_t level, void* h_buf, int64_t* len) {
  if (!h || !len) {
    g_last_error = "bad arguments";
    return MGM_E_ARG;
  }
  return guard([&] {
    const HostHierarchy& H = h->H;
    const int p = int(H.lv.size());
    auto need_level = [&](int maxl) {
      if (level < 0 || level > maxl) throw Error(MGM_E_ARG, "level out of range");
    };
    std::vector<int32_t> vi;
    std::vector<double> vd;
    bool isint = true;
    switch (what) {
      case MGM_EX_LEVEL_SIZES:
        for (auto& l : H.lv) vi.push_back(l.n);
        break;
      case MGM_EX_STENCILS: vi = H.stencils; break;
      case MGM_EX_WEIGHTS: vd = H.weights; isint = false; break;
      case MGM_EX_COARSE_IDX: need_level(p - 2); vi = H.lv[level].coarse_idx; break;
      case MGM_EX_INTERP_IDX: need_level(p - 2); vi = H.lv[level].pidx; break;
      case MGM_EX_INTERP_W: need_level(p - 2); vd = H.lv[level].pw; isint = false; break;
      case MGM_EX_COLOURS: need_level(p - 2); vi = H.lv[level].colour; break;
      case MGM_EX_L_ROWPTR: need_level(p - 1); vi = H.lv[level].L.ptr; break;
      case MGM_EX_L_COLS: need_level(p - 1); vi = H.lv[level].L.col; break;
      case MGM_EX_L_VALS: need_level(p - 1); vd = H.lv[level].L.val; isint = false; break;
      case MGM_EX_BORDER: need_level(p - 1); vd = H.lv[level].b; isint = false; break;
      case MGM_EX_PATCH: need_level(p - 2); vi = H.lv[level].patch; break;
      case MGM_EX_GRAD_STENCILS: vi = h->sg_sten; break;
      case MGM_EX_GRAD_WEIGHTS: vd = h->sg_w; isint = false; break;
      case MGM_EX_OMEGA: {
        need_level(p - 2);
        if (level >= int(h->ls.size()) || !h->ls[level].om64) throw Error(MGM_E_ARG, "learned smoother not trained");
        const int n = h->lv[level].n, s = h->ls[level].s;
        std::vector<double> om(size_t(n) * s);
        std::vector<int32_t> perm(n);
        HIPCHECK(hipMemcpy(om.data(), h->ls[level].om64, om.size() * sizeof(double), hipMemcpyDeviceToHost));
        if (h->lv[level].perm) HIPCHECK(hipMemcpy(perm.data(), h->lv[level].perm, n * sizeof(int32_t), hipMemcpyDeviceToHost));
        else std::iota(perm.begin(), perm.end(), 0);
        vd.assign(size_t(n) * s, 0.0);
        for (int q = 0; q < s; ++q)
          for (int pos = 0; pos < n; ++pos) vd[size_t(perm[pos]) * s + q] = om[size_t(q) * n + pos];
        isint = false;
        break;
      }
      case MGM_EX_NCOLOURS:
        for (int j = 0; j + 1 < p; ++j) vi.push_back(H.lv[j].ncolours);
        break;
      case MGM_EX_L16_VALS:
      case MGM_EX_ROW_SCALE: {
        // the FP16 operator the device holds (built on first use), read back
        // and moved from the device's permuted numbering to the natural one
        need_level(p - 2);
        need_device(h);
        HIPCHECK(hipSetDevice(h->device));
        build_precision(h, MGM_FP16);
        const DevLevel& d = h->lv[level];
        const Csr& L = H.lv[level].L;
        const int n = d.n;
        std::vector<int32_t> perm(n), rp(n + 1);
        if (d.perm) HIPCHECK(hipMemcpy(perm.data(), d.perm, n * sizeof(int32_t), hipMemcpyDeviceToHost));
        else std::iota(perm.begin(), perm.end(), 0);
        HIPCHECK(hipMemcpy(rp.data(), d.rowptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
        const int64_t nnz = rp[n];
        if (nnz != int64_t(L.val.size())) throw Error(MGM_E_ARG, "device operator pattern differs from the host's");
        if (what == MGM_EX_ROW_SCALE) {
          std::vector<float> sc(n);
          HIPCHECK(hipMemcpy(sc.data(), d.s16, n * sizeof(float), hipMemcpyDeviceToHost));
          vd.assign(n, 0.0);
          for (int pos = 0; pos < n; ++pos) vd[perm[pos]] = double(sc[pos]);
        } else {
          std::vector<int32_t> cl(nnz);
          std::vector<_Float16> hv(nnz);
          HIPCHECK(hipMemcpy(cl.data(), d.col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
          HIPCHECK(hipMemcpy(hv.data(), d.v16, nnz * sizeof(_Float16), hipMemcpyDeviceToHost));
          vd.assign(nnz, std::nan(""));
          for (int pos = 0; pos < n; ++pos) {
            const int i = perm[pos];
            const int32_t* c0 = L.col.data() + L.ptr[i];
            const int32_t* c1 = L.col.data() + L.ptr[i + 1];
            for (int k = rp[pos]; k < rp[pos + 1]; ++k) {
              const int32_t cn = perm[cl[k]];
              const int32_t* at = std::lower_bound(c0, c1, cn);
              if (at == c1 || *at != cn) throw Error(MGM_E_ARG, "device operator pattern differs from the host's");
              vd[size_t(at - L.col.data())] = double(float(hv[k]));
            }
          }
        }
        isint = false;
        break;
      }
      case MGM_EX_HALO_ROWS: {
        // the staged halo lists of the one-launch sweeps, moved from the
        // device's slot order and permuted numbering to patch ids and the
        // natural numbering
        need_level(p - 2);
        need_device(h);
        HIPCHECK(hipSetDevice(h->device));
        const DevLevel& d = h->lv[level];
        if (!d.patched || !d.halo_ok) break;
        const int n = d.n, nsl = d.pstart_host_slots;
        std::vector<int32_t> perm(n), ps(nsl + 1), hs(nsl + 1);
        if (d.perm) HIPCHECK(hipMemcpy(perm.data(), d.perm, n * sizeof(int32_t), hipMemcpyDeviceToHost));
        else std::iota(perm.begin(), perm.end(), 0);
        HIPCHECK(hipMemcpy(ps.data(), d.pstart, (nsl + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(hs.data(), d.fl_hstart, (nsl + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::vector<int32_t> hr(std::max(hs[nsl], 1));
        HIPCHECK(hipMemcpy(hr.data(), d.fl_hrows, hr.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        const std::vector<int32_t>& patch = H.lv[level].patch;
        std::vector<std::vector<int32_t>> lists(size_t(H.lv[level].npatch));
        for (int sl = 0; sl < nsl; ++sl) {
          if (ps[sl + 1] <= ps[sl]) continue;
          auto& l = lists[size_t(patch[perm[ps[sl]]])];
          for (int k = hs[sl]; k < hs[sl + 1]; ++k) l.push_back(perm[hr[k]]);
          std::sort(l.begin(), l.end());
        }
        for (const auto& l : lists) {
          vi.push_back(int32_t(l.size()));
          vi.insert(vi.end(), l.begin(), l.end());
        }
        break;
      }
      default: throw Error(MGM_E_ARG, "unknown export item");
    }
    int64_t cnt = isint ? int64_t(vi.size()) : int64_t(vd.size());
    if (h_buf) {
      if (*len < cnt) throw Error(MGM_E_ARG, "export buffer too small");
      if (isint) std::memcpy(h_buf, vi.data(), cnt * sizeof(int32_t));
      else std::memcpy(h_buf, vd.data(), cnt * sizeof(double));
    }
    *len = cnt;
  });
}

void mgm_destroy(mgm_handle h) {
  if (!h) return;
  if (h->device >= 0) {
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (int k = 0; k < 3; ++k)
      if (h->graph[k]) (void)hipGraphExecDestroy(h->graph[k]);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (void* p : h->allocs) (void)hipFree(p);
    if (h->hpin) (void)hipHostFree(h->hpin);
    if (h->hflow_err) (void)hipHostFree(h->hflow_err);
    if (h->step_done) (void)hipEventDestroy(h->step_done);
  }
  delete h;
}

const char* mgm_status_str(mgm_status s) {
  switch (s) {
    case MGM_OK: return "ok";
    case MGM_NOT_CONVERGED: return "not converged";
    case MGM_E_ARG: return "invalid argument";
    case MGM_E_ALLOC: return "allocation failed";
    case MGM_E_HIP: return "HIP error";
    case MGM_E_STENCIL_SINGULAR: return "singular stencil system";
    case MGM_E_DUP_POINTS: return "duplicate points";
    case MGM_E_ZERO_DIAG: return "zero diagonal";
    case MGM_E_COARSE_SINGULAR: return "singular coarse operator";
    case MGM_E_BREAKDOWN: return "Krylov breakdown";
    case MGM_E_NONFINITE: return "non-finite value";
    case MGM_E_SYNC: return "smoother sweep synchronisation failed";
  }
  return "unknown status";
}

const char* mgm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
