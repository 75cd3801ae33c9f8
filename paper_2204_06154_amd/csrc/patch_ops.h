// Whole-level row operators that read the operator from the patch ELL of a
// patch-blocked level (the smoother's storage): one workgroup per half patch
// slot (kRowHalf rows), kPatchG lanes per row, so every entry load of a
// workgroup covers 512 consecutive elements and the operator streams at full
// width. Half slots give twice as many workgroups as slots, so the last round
// of workgroups on the chip is short (with one per slot, 625 slots of the
// fine torus level ran as three rounds of 256 for 2.4 rounds of work).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs_patch.h"
#include "lane_ops.h"

namespace mgm {
namespace {

// MODE kRowResidual: out = f - A x (SCALED: A = diag(scale) H), minus
//   b_i * (*lam) when BORDER, and with BDOT partial[slot] = sum over the
//   slot's rows of b_i x_i (fixed tree).
// MODE kRowApply:   out = A x, plus b_i * (*lam) when BORDER (the bordered
//   operator's multiplier column); with BDOT the partial sums of b_i x_i as
//   above (its constraint row).
// MODE kRowRichardson: out = x + omega_i dinv_i (f - A x), one step of the
//   learned per-node smoother (out and x distinct); with BORDER the
//   multiplier is held fixed, f - A x - b_i * (*lam).
constexpr int kRowResidual = 0;
constexpr int kRowApply = 1;
constexpr int kRowRichardson = 2;
// x may be stored in a narrower type X than the arithmetic type S; with xcopy
// given, every row also writes S(x_i) there (and, bordered, xcopy[tail] =
// *lam): the FGMRES step uses this to widen the preconditioner's FP32 output
// while applying the operator to it.
constexpr int kRowHalf = kPatch / 2;
template <typename V, typename S, typename X, int WL, bool SCALED, int MODE, bool BDOT, bool BORDER>
__global__ __launch_bounds__(kRowHalf * kPatchG) void k_rowop_patch(
    int nw, int block, const int32_t* __restrict__ pstart, const V* __restrict__ pval,
    const int32_t* __restrict__ pcol, const float* __restrict__ scale, const S* __restrict__ f,
    const X* __restrict__ x, S* __restrict__ out, const S* __restrict__ b, const double* __restrict__ lam,
    double* __restrict__ partial, const S* __restrict__ dinv, const S* __restrict__ omega,
    S* __restrict__ xcopy, int tail) {
  const int slot = blockIdx.x >> 1;
  const int t = (blockIdx.x & 1) * kRowHalf + int(threadIdx.x) / kPatchG;
  const int g = threadIdx.x % kPatchG;
  const bool slot_row = t < block;
  const int tt = slot_row ? t : 0;  // lanes past the slot's rows read row 0's entries (in bounds, unused)
  const int64_t base = (int64_t(slot) * block * nw + tt) * kPatchG + g;
  int cc[WL];
  S iv[WL];
#pragma unroll
  for (int i = 0; i < WL; ++i) {
    const int ii = i < nw ? i : nw - 1;
    const int64_t e = base + int64_t(ii) * block * kPatchG;
    // unconditional loads: no branch forces a wait between them
    const int32_t cv = pcol[e];
    const V vv = pval[e];
    cc[i] = cv;
    iv[i] = (slot_row && i < nw) ? S(vv) : S(0);
  }
  const int r0 = pstart[slot];
  const int nr = pstart[slot + 1] - r0;
  const bool act = t < nr;
  const int row = r0 + t;
  // The slot's own rows are a contiguous range of x: stage it (both halves'
  // rows) in LDS and take the in-patch columns (most of them) from there; only
  // the halo columns go to the cache hierarchy, and those loads are issued
  // before the barrier.
  __shared__ S xl[kPatch];
  for (int q = int(threadIdx.x); q < nr; q += int(blockDim.x)) xl[q] = S(x[r0 + q]);
  if (xcopy && act && g == 0) xcopy[row] = S(x[row]);
  if (BORDER && xcopy && blockIdx.x == 0 && threadIdx.x == 0) xcopy[tail] = S(*lam);
  // Halo gathers are issued unconditionally, so that no branch makes a load
  // wait for the one before it; in-patch and padding entries read the row's
  // own value instead (one cache line) and are masked out of the sums. Each
  // sum adds the same terms in the same order as a masked loop would.
  S a0 = S(0), a1 = S(0);
  if (act) {
    X xv[WL];
#pragma unroll
    for (int i = 0; i < WL; ++i) {
      const bool halo = i < nw && unsigned(cc[i] - r0) >= unsigned(nr);
      xv[i] = x[halo ? cc[i] : row];
    }
#pragma unroll
    for (int i = 0; i < WL; i += 2) {
      if (i < nw && unsigned(cc[i] - r0) >= unsigned(nr)) a0 += iv[i] * S(xv[i]);
      if (i + 1 < WL && i + 1 < nw && unsigned(cc[i + 1] - r0) >= unsigned(nr)) a1 += iv[i + 1] * S(xv[i + 1]);
    }
  }
  __syncthreads();
  if (act) {
    S lv[WL];
#pragma unroll
    for (int i = 0; i < WL; ++i) lv[i] = xl[unsigned(cc[i] - r0) < unsigned(nr) ? cc[i] - r0 : 0];
#pragma unroll
    for (int i = 0; i < WL; i += 2) {
      if (i < nw && unsigned(cc[i] - r0) < unsigned(nr)) a0 += iv[i] * lv[i];
      if (i + 1 < WL && i + 1 < nw && unsigned(cc[i + 1] - r0) < unsigned(nr)) a1 += iv[i + 1] * lv[i + 1];
    }
  }
  S acc = group_sum<kPatchG>(a0 + a1);
  double bx = 0.0;
  if (act && g == 0) {
    if (SCALED) acc *= S(scale[row]);
    if (MODE == kRowResidual) {
      if (BORDER) acc += b[row] * S(*lam);  // continuing iterate: f - A x - b lambda
      out[row] = f[row] - acc;
      if (BDOT) bx = double(b[row]) * double(xl[t]);
    } else if (MODE == kRowRichardson) {
      if (BORDER) acc += b[row] * S(*lam);  // multiplier held fixed: f - A x - b lambda
      out[row] = xl[t] + omega[row] * dinv[row] * (f[row] - acc);
    } else {
      if (BORDER) acc += b[row] * S(*lam);
      out[row] = acc;
      if (BDOT) bx = double(b[row]) * double(xl[t]);  // the bordered constraint row b . x
    }
  }
  if (BDOT) {  // one partial per workgroup (two per slot)
    __shared__ double sh[kRowHalf * kPatchG];
    sh[threadIdx.x] = bx;
    __syncthreads();
    for (int s = kRowHalf * kPatchG / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
  }
}

}  // namespace
}  // namespace mgm
