// Patch-blocked multicolour Gauss-Seidel sweep kernel for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include "lane_ops.h"

namespace mgm {
namespace {

// Patch-blocked Gauss-Seidel: one workgroup sweeps one patch (<= kPatch rows)
// of the current patch colour, kPatchG consecutive lanes per row. Patches of
// one colour never couple, so the values outside the patch ("halo") are
// constant during the launch: the lanes of a row fold its halo entries into
// the right-hand side once, keep the in-patch entries (value, local column)
// in registers, and the patch values live in LDS. The local colours are then
// visited in order (reverse for a backward sweep), one barrier each: rows of
// one local colour never couple, so this is sequential GS in the order
// (patch colour, patch, local colour).
// With zero_guess the sweep starts from u = 0 without reading u: rows of patch
// colours visited earlier in this sweep hold their new values, all others are
// taken as zero (so no separate clearing pass is needed).
// Operator storage per patch slot: ELL with the level's width nw * kPatchG
// and a fixed stride of `block` rows, entry i*kPatchG + g of local row t at
// (slot * block * nw + i * block + t) * kPatchG + g, so the lanes of a
// workgroup read consecutive addresses and the entry loads depend on no other
// load; padding entries have value zero and a valid column.
//
// Dataflow variant (FLOW): one launch sweeps every patch colour of the level.
// A patch may start once every coupled patch that precedes it in the sweep
// order has finished (it reads their new values, and they must have read its
// old ones), so the sweep is the same sequential GS order without a launch
// boundary per colour. Workgroups take their position in the sweep order from
// a ticket counter, so a workgroup only waits for workgroups that are already
// running or done (no deadlock whatever the dispatch order); the counter is
// never reset, and ticket / slots + 1 numbers the sweep, which is what each
// patch's flag records when it finishes. Values that pass between workgroups
// of the launch (the final stores of u, the halo loads, the flags) are
// agent-scope atomic accesses, which the hardware keeps coherent across the
// chip's L2 caches (stores written through, loads not served from a stale
// line); a wave waits for its stores to complete before the barrier that
// precedes the flag store, and the halo loads are issued after the barrier
// that follows the wait, so no cache write-back or invalidation is needed.
// A wait gives up after fl.wait_ticks ticks of the constant-rate real-time
// counter (by default kFlowWaitTicks = 2^24: ~0.17 s at its usual 100 MHz,
// against waits of tens of microseconds) and raises the error flag, so every
// workgroup ends; the host then resets the level's ticket counter and flags.
constexpr int kPatch = 256;
constexpr int kPatchG = 4;
constexpr unsigned long long kFlowWaitTicks = 1ull << 24;
// s_waitcnt operand (gfx9 encoding) for vmcnt(0) with expcnt and lgkmcnt left
// at their maxima: wait for this wave's outstanding vector memory operations
constexpr int kWaitVmcnt0 = 0x0F70;

struct GsFlow {
  unsigned long long* ticket;    // sweeps * slots workgroups started so far
  unsigned* flag;                // per slot: number of the last sweep it finished
  const int32_t* nbptr;          // coupled slots of slot s: nb[nbptr[s] .. nbptr[s+1])
  const int32_t* nb;
  const int32_t* crow;           // slot s: rows [crow[2s], crow[2s+1]) of its patch colour
  int* err;                      // set when a wait gave up
  int nslot;
  unsigned long long wait_ticks;  // bound of each wait (real-time counter ticks)
  const int32_t* hstart;         // staged halo: slot s reads rows hrows[hstart[s] .. hstart[s+1])
  const int32_t* hrows;
};

// Staged halo (HALO, one-launch sweeps): the distinct rows outside a patch
// that its entries reference (a few hundred, against a few thousand entries)
// are listed per slot in ascending order; the workgroup loads each of them
// once into LDS, with consecutive lanes on consecutive rows (rows of slots
// later in the sweep before the wait, the others after it), and the lanes
// gather their out-of-patch values from there. The column array then holds
// the in-patch row (below kPatch) or kPatch + the row's place in the slot's
// list. Same values, same sums: results are those of the direct loads.
constexpr int kMaxHalo = kPatch * kPatchG;  // staged rows per slot (one per thread)
// With 32-bit vectors a level stages its halo only if it has at most this many
// patch slots: on larger levels, whose workgroups outnumber what the chip
// holds at once, the per-entry loads measured faster for 4-byte values (FP64
// vectors stage on every level).
constexpr int kStageMaxSlots = 512;

template <typename V, typename S, int WL, bool SCALED, bool BORDER, bool FLOW = false, bool HALO = false>
__global__ __launch_bounds__(kPatch * kPatchG) void k_gs_patch(
    int slot0, int reverse, int zero_guess, int nw, int block, const int32_t* __restrict__ pstart,
    const int32_t* __restrict__ pncl, const int32_t* __restrict__ lcol,
    const V* __restrict__ pval, const int32_t* __restrict__ pcol, const float* __restrict__ scale,
    const S* __restrict__ dinv, const S* __restrict__ f, S* u, const S* __restrict__ b,
    const double* __restrict__ lam, GsFlow fl) {
  static_assert(!HALO || FLOW, "staged halo: one-launch sweeps");
  __shared__ S ul[kPatch];
  __shared__ S hv[HALO ? kMaxHalo : 1];
  __shared__ unsigned s_ticket[2];
  int slot = slot0 + blockIdx.x;
  unsigned sweep = 0;
  if (FLOW) {
    if (threadIdx.x == 0) {
      const unsigned long long tk =
          __hip_atomic_fetch_add(fl.ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_ticket[0] = unsigned(tk % unsigned(fl.nslot));
      s_ticket[1] = unsigned(tk / unsigned(fl.nslot)) + 1u;
    }
    __syncthreads();
    slot = reverse ? fl.nslot - 1 - int(s_ticket[0]) : int(s_ticket[0]);
    sweep = s_ticket[1];
  }
  const int t = threadIdx.x / kPatchG;
  const int g = threadIdx.x % kPatchG;
  const bool slot_row = t < block;
  const int tt = slot_row ? t : 0;  // lanes past the slot's rows read row 0's entries (in bounds, unused)
  // entry loads first: their addresses need no other load
  const int64_t base = (int64_t(slot) * block * nw + tt) * kPatchG + g;
  int cc[WL];
  S iv[WL];
#pragma unroll
  for (int i = 0; i < WL; ++i) {
    const int ii = i < nw ? i : nw - 1;  // chunks >= nw: re-read the last one, zeroed below
    const int64_t e = base + int64_t(ii) * block * kPatchG;
    // unconditional loads: no branch forces a wait between them
    const int32_t cv = pcol[e];
    const V vv = pval[e];
    cc[i] = cv;
    iv[i] = (slot_row && i < nw) ? S(vv) : S(0);
  }
  const int r0 = pstart[slot];
  const int nr = pstart[slot + 1] - r0;
  const int ncl = pncl[slot];
  int hrow = 0;
  bool hact = false;
  if (HALO) {
    // this thread's staged row (the list is known before the wait)
    const int h0 = fl.hstart[slot];
    hact = int(threadIdx.x) < fl.hstart[slot + 1] - h0;
    if (hact) hrow = fl.hrows[h0 + int(threadIdx.x)];
  }
  // rows [upd_lo, upd_hi) hold current values (all rows unless zero_guess)
  int upd_lo = 0, upd_hi = INT_MAX;
  if (zero_guess) {
    if (FLOW) {
      if (reverse) upd_lo = fl.crow[2 * slot + 1];
      else upd_hi = fl.crow[2 * slot];
    } else {
      if (reverse) upd_lo = pstart[slot0 + gridDim.x];
      else upd_hi = pstart[slot0];
    }
  }
  const bool act = t < nr;
  const int row = r0 + t;
  // staged rows of slots after this one in the sweep keep their old values
  // until this patch is done (those slots wait for it): load them before the wait
  S hval = S(0);
  bool hlate = false;
  if (HALO && hact) {
    hlate = reverse ? hrow < r0 : hrow > r0;
    if (hlate && hrow >= upd_lo && hrow < upd_hi)
      hval = __hip_atomic_load(u + hrow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  int ic[WL];
  S rhs = S(0), di = S(0), sc = S(1), uown = S(0);
  int myc = -1;
  if (act) {
    uown = zero_guess ? S(0) : u[row];
    myc = lcol[row];
    di = dinv[row];
    rhs = f[row];
    if (SCALED) sc = S(scale[row]);
    if (BORDER) rhs -= b[row] * S(*lam);
  }
  if (FLOW) {
    // the first wave waits for the coupled slots that precede this one
    if (threadIdx.x < 64) {
      const int k1 = fl.nbptr[slot + 1];
      for (int k = fl.nbptr[slot] + int(threadIdx.x); k < k1; k += 64) {
        const int q = fl.nb[k];
        if (reverse ? q > slot : q < slot) {
          const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
          while (int(__hip_atomic_load(fl.flag + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - sweep) < 0) {
            if (__builtin_amdgcn_s_memrealtime() - t0 > fl.wait_ticks) {
              __hip_atomic_store(fl.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
      }
    }
    __syncthreads();
  }
  if (HALO) {
    if (hact) {
      if (!hlate && hrow >= upd_lo && hrow < upd_hi)
        hval = __hip_atomic_load(u + hrow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      hv[threadIdx.x] = hval;
    }
    __syncthreads();
  }
  if (act) {
    S halo = S(0);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
      const bool live = i < nw;
      if (HALO) {
        // cc: in-patch row, or kPatch + place in the staged list
        const bool in = live && cc[i] < kPatch;
        const S hx = hv[(live && !in) ? cc[i] - kPatch : 0];
        halo += iv[i] * ((live && !in) ? hx : S(0));
        ic[i] = in ? cc[i] : t;
        iv[i] = in ? iv[i] : S(0);
        continue;
      }
      const bool in = live && unsigned(cc[i] - r0) < unsigned(nr);
      const bool cur = cc[i] >= upd_lo && cc[i] < upd_hi;
      S uv = S(0);
      if (FLOW) {
        // agent-coherent load: the value another workgroup wrote through in this launch
        if (live && !in && cur) uv = __hip_atomic_load(u + cc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uv = (live && !in && cur) ? u[cc[i]] : S(0);
      }
      halo += iv[i] * uv;
      ic[i] = in ? cc[i] - r0 : t;
      iv[i] = in ? iv[i] : S(0);
    }
    halo = group_sum<kPatchG>(halo);
    rhs -= sc * halo;
    if (g == 0) ul[t] = uown;
  }
  __syncthreads();
  // Each row keeps its own value in a register (only that row writes it).
  for (int step = 0; step < ncl; ++step) {
    const int c = reverse ? ncl - 1 - step : step;
    if (myc == c) {  // all lanes of a row agree
      S a[4] = {S(0), S(0), S(0), S(0)};
#pragma unroll
      for (int i = 0; i < WL; ++i) a[i & 3] += iv[i] * ul[ic[i]];
      // issue every LDS gather of the step before the first multiply-add (one
      // LDS latency per step instead of one per batch of eight)
      __builtin_amdgcn_sched_group_barrier(0x100, WL, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 4 * WL, 0);
      const S acc = group_sum<kPatchG>((a[0] + a[1]) + (a[2] + a[3]));
      uown = uown + (rhs - sc * acc) * di;
      if (g == 0) ul[t] = uown;
    }
    __syncthreads();
  }
  if (FLOW) {
    // agent-coherent (write-through) stores; each wave waits for its own to
    // complete before the barrier, after which the flag is raised
    if (act && g == 0) __hip_atomic_store(u + row, uown, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(fl.flag + slot, sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if (act && g == 0) {
    u[row] = uown;
  }
}

}  // namespace
}  // namespace mgm
