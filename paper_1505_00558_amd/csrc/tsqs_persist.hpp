// tsqs_persist.hpp -- the persistent schedule: one kernel whose workgroups take
// tasks from a ring in device memory until no key is left to place.
//
// It finishes every sort (the parts left after the level schedule's passes,
// and the parts that wait for an exact pivot), and it runs a whole batch in
// one launch when the persistent schedule is chosen.  Tasks:
//   kTaskPart    chunks [c0, c1) of a pool part to partition (the level
//                kernels' chunk code, one- or two-level by the part's flags);
//                the workgroup that finishes the part's last chunk plans it:
//                equal bands (long ones become band tasks), small children
//                listed for k_finish_list (the launch after this kernel),
//                large children become pool parts with tasks;
//   kTaskSelect  chunks [c0, c1) of a part whose exact pivot is being
//                selected: one 8-bit radix digit per round, histograms in LDS
//                added into the part's global histogram; the workgroup that
//                finishes a round fixes the digit and starts the next round,
//                or, after the last digit, the part's partition (the
//                guaranteed fallback of the depth limit, spread over the grid);
//   kTaskBand    one kBandChunk piece of a long band.
// A workgroup claims ring indices in order (one atomic); a claimed slot not yet
// written is waited for while keys remain.  Nothing waits for a given
// workgroup, so the workgroups need not be resident together (no cooperative
// launch).  The kernel ends when the count of keys not yet final reaches zero;
// a workgroup that exceeds the iteration cap, or a full ring or pool, sets an
// error flag and every workgroup leaves at its next claim.
#pragma once

#include "tsqs_kernels.hpp"

namespace tsqs {

enum { kStTailParts = 6, kStTailKeys = 7, kStSelRounds = 8 };

// Control area of a persistent workgroup's LDS (the rest is shared by the
// phases: partition stage, plan, select histogram).
struct PersistCtl {
  Task task;
  uint32_t state;        // 0 a task, 1 no keys left, 2 abort
  uint32_t last;         // this workgroup finished the last chunk of a phase
  uint32_t final_keys;   // keys the plan took out of this kernel's count (final or listed)
  uint32_t pad;
};
constexpr size_t kPCtlBytes = 256;
static_assert(sizeof(PersistCtl) <= kPCtlBytes, "control area");

// Dynamic LDS of k_persist for key type DT.
template <int DT, bool HASV>
constexpr size_t persist_lds() {
  size_t a = sizeof(PartLds<DT, HASV, false, kPNT>);
  if (sizeof(PartLds<DT, HASV, true, kPNT>) > a) a = sizeof(PartLds<DT, HASV, true, kPNT>);
  if ((size_t)kPNW * 256 * 4 > a) a = (size_t)kPNW * 256 * 4;
  return kPCtlBytes + a;
}

// Parts of level d become pool parts with their partition tasks (a wave per part).
template <int DT, bool HASV>
__global__ __launch_bounds__(kPlanNT) void k_seed(Ctx c, int d) {
  const unsigned long long packed = c.lvl[d].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  if (nseg == 0 || nseg > c.seg_cap) return;
  const Seg *segs = (d & 1) ? c.seg1 : c.seg0;
  const uint32_t wv = threadIdx.x / kWave, lane = threadIdx.x & 63u;
  for (uint32_t i = blockIdx.x * kPlanNW + wv; i < nseg; i += gridDim.x * kPlanNW) {
    TPart tp;
    tp.s = segs[i];
    tp.s.chunk_begin = 0;
    uint32_t id = ~0u;
    if (lane == 0) {
      const unsigned long long pid = atomicAdd(&c.p.ctl[kQParts], 1ull);
      if (pid < c.p.part_cap) id = (uint32_t)pid;
      else persist_abort(c, kErrQueue);
    }
    id = shfl_u32(id, 0);
    if (id == ~0u) return;
    tp.nchunks = pool_chunks<DT, HASV>(c, tp.s.off, tp.s.len, tp.s.flags);
    tp.done = 0; tp.round = 0; tp.krem = 0; tp.prefix = 0; tp.mask = 0; tp.hslot = 0; tp.pad = 0;
    pool_put(c, id, tp);
    if (lane == 0) atomicAdd(&c.p.ctl[kQLeft], (unsigned long long)tp.s.len);
    pool_tasks(c, id, kTaskPart, tp.nchunks);
  }
}

// A child of a planned part (one wave): small ones are listed for
// k_finish_list, large ones become pool parts (with their tasks, or their
// selection if the depth limit asks for the exact median).
template <int DT, bool HASV>
__device__ inline void persist_child(const Ctx &c, PersistCtl &P, uint64_t off, uint32_t len,
                                     uint32_t depth, uint32_t dmax, uint32_t req, bool in_s,
                                     uint64_t own, unsigned long long look, uint32_t *hist) {
  using B = typename Codec<DT>::B;
  const uint32_t lane = lane_id();
  if (len <= c.small_max) {
    if (lane == 0 && len > 0) {
      if (len > 1 || in_s) {
        FinItem it;
        it.off = off; it.src = 0; it.pivot = 0; it.len = len;
        it.kind = (in_s ? 2u : 0u) | (req << 2);
        const bool wave = next_pow2(len) <= c.wave_max;
        const unsigned long long x = atomicAdd(&c.p.ctl[wave ? kQFinw : kQFin], 1ull);
        const unsigned long long y = __hip_atomic_load(&c.p.ctl[wave ? kQFin : kQFinw], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        if (x + y < c.p.sfin_cap) c.p.sfin[wave ? c.p.sfin_cap - 1 - x : x] = it;
        else persist_abort(c, kErrQueue);
        stat_add(c, kStSmallParts, 1ull);
        stat_add(c, kStSmallKeys, len);
      } else if (c.dbg) {
        dbg_final(c, off);   // one key already in K: final in place
      }
      atomicAdd(&P.final_keys, len);
    }
    return;
  }
  const B *Y = (const B *)(in_s ? c.S : c.K);
  uint32_t S = c.samples;
  if (S > len) S = (len & 1) ? len : len - 1;
  const uint32_t nlt = (uint32_t)look, neq = (uint32_t)(look >> 32);
  const bool exact = c.pivot_mode == 1 || depth >= dmax;
  const bool fits = (uint64_t)nlt + neq <= len;
  if (!fits && lane == 0) atomicOr(c.err, kErrCount);
  const bool two = !exact && fits;
  B p0 = (B)own;
  if (exact) {
    const uint32_t kk = (c.pivot_mode == 1 && depth < dmax) ? 0u : len / 2;
    if (lane == 0 && depth >= dmax) stat_add(c, kStFallback, 1ull);
    if (len > kSelInline && start_select(c, off, len, depth, dmax, req, in_s, kk, false)) return;
    p0 = wave_select<DT>(Y, off, len, kk, hist);
  }
  uint64_t piv[7];
  wave_part_pivots<DT>(Y, off, len, S, c.jitter, true, p0, piv);
  uint32_t id = ~0u;
  if (lane == 0) {
    const unsigned long long pid = atomicAdd(&c.p.ctl[kQParts], 1ull);
    if (pid < c.p.part_cap) id = (uint32_t)pid;
    else persist_abort(c, kErrQueue);
  }
  id = shfl_u32(id, 0);
  if (id == ~0u) return;
  TPart tp;
  tp.s.off = off;
#pragma unroll
  for (int q = 0; q < 7; q++) tp.s.piv[q] = piv[q];
  tp.s.len = len; tp.s.chunk_begin = 0; tp.s.depth = depth; tp.s.dmax = dmax; tp.s.req = req;
  tp.s.flags = (in_s ? kSegInS : 0u) | (two ? kSegTwo : 0u);
  tp.s.nlt = two ? nlt : 0u;
  tp.s.neq = two ? neq : 0u;
  tp.nchunks = pool_chunks<DT, HASV>(c, off, len, tp.s.flags);
  tp.done = 0; tp.round = 0; tp.krem = 0; tp.prefix = 0; tp.mask = 0; tp.hslot = 0; tp.pad = 0;
  pool_put(c, id, tp);
  pool_tasks(c, id, kTaskPart, tp.nchunks);
}

// Plans pool part id after its partition (whole workgroup).
template <int DT, bool HASV, bool DBG>
__device__ void persist_plan(const Ctx &c, PersistCtl &P, unsigned char *area, uint32_t id) {
  const uint32_t tid = threadIdx.x, wv = tid >> 6, lane = tid & 63u;
  const Seg s = c.p.parts[id].s;
  const unsigned long long *cp = c.p.pctr + (size_t)id * kCtrStride;
  const bool out_s = (s.flags & kSegInS) == 0;   // children live in the other buffer
  uint64_t coff[4] = {0, 0, 0, 0}, cown[4] = {0, 0, 0, 0};
  uint32_t clen[4] = {0, 0, 0, 0};
  unsigned long long clook[4] = {0, 0, 0, 0};
  FinItem band[3];
  int nch = 0;
  uint32_t cdepth = 0;
  for (int b = 0; b < 3; b++) { band[b].off = 0; band[b].src = 0; band[b].pivot = 0; band[b].len = 0; band[b].kind = s.req << 2; }
  if (s.flags & kSegTwo) {
    const unsigned long long ca = __hip_atomic_load(cp + kCtrA, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long cb = __hip_atomic_load(cp + kCtrB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t nll = (uint32_t)ca, nlg = (uint32_t)(ca >> 32);
    const uint32_t ngl = (uint32_t)cb, ngg = (uint32_t)(cb >> 32);
    const uint32_t nlt = s.nlt, neq = s.neq, g0 = nlt + neq;
    if ((uint64_t)nll + nlg > nlt || (uint64_t)g0 + ngl + ngg > s.len) {
      if (tid == 0) persist_abort(c, kErrCount);
      return;
    }
    const uint32_t ele = nlt - nll - nlg, egt = (s.len - g0) - ngl - ngg;
    // payloads of each band were staged at [0, ...), [nlt, ...), [g0, ...)
    band[0].off = s.off + nll; band[0].src = s.off; band[0].len = ele; band[0].pivot = s.piv[1];
    band[1].off = s.off + nlt; band[1].src = s.off + nlt; band[1].len = neq; band[1].pivot = s.piv[0];
    band[2].off = s.off + g0 + ngl; band[2].src = s.off + g0; band[2].len = egt; band[2].pivot = s.piv[2];
    coff[0] = s.off; coff[1] = s.off + nlt - nlg; coff[2] = s.off + g0; coff[3] = s.off + s.len - ngg;
    clen[0] = nll; clen[1] = nlg; clen[2] = ngl; clen[3] = ngg;
    nch = 4;
    cdepth = 2;   // recursion levels from the part to its children
    for (int k = 0; k < 4; k++) {
      cown[k] = s.piv[3 + k];
      clook[k] = __hip_atomic_load(cp + kCtrLook + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else {
    const unsigned long long cv = __hip_atomic_load(cp + kCtrA, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t L = (uint32_t)cv, G = (uint32_t)(cv >> 32);
    if ((uint64_t)L + G > s.len) {
      if (tid == 0) persist_abort(c, kErrCount);
      return;
    }
    band[1].off = s.off + L; band[1].src = s.off; band[1].len = s.len - L - G; band[1].pivot = s.piv[0];
    coff[0] = s.off; clen[0] = L; cown[0] = s.piv[1];
    coff[1] = s.off + s.len - G; clen[1] = G; cown[1] = s.piv[2];
    clook[0] = __hip_atomic_load(cp + kCtrLook + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    clook[1] = __hip_atomic_load(cp + kCtrLook + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    nch = 2;
    cdepth = 1;
  }
  if (tid == 0) {
    P.final_keys = 0;
    stat_add(c, kStTailParts, 1ull);
    stat_add(c, kStTailKeys, s.len);
  }
  __syncthreads();
  // bands: short ones written now by the workgroup, long ones as band tasks
  uint32_t band_now = 0;
  for (int b = 0; b < 3; b++) {
    if (band[b].len == 0) continue;
    if (band[b].len <= kBandChunk) {
      fill_band<DT, HASV, DBG>(c, band[b], tid, kPNT);
      band_now += band[b].len;
    } else if (wv == 0) {
      uint32_t bid = ~0u;
      if (lane == 0) {
        const unsigned long long x = atomicAdd(&c.p.ctl[kQBands], 1ull);
        if (x < c.p.band_cap) { bid = (uint32_t)x; c.p.bands[bid] = band[b]; }
        else persist_abort(c, kErrQueue);
      }
      bid = shfl_u32(bid, 0);
      if (bid != ~0u) {
        const uint32_t pieces = (band[b].len + kBandChunk - 1) / kBandChunk;
        push_tasks(c, pieces, [&](uint32_t i) {
          Task t; t.kind = kTaskBand; t.id = bid; t.c0 = i; t.c1 = i + 1; return t;
        });
      }
    }
    if (tid == 0) stat_add(c, kStBandKeys, band[b].len);
  }
  // children: wave k takes child k
  uint32_t *hist = reinterpret_cast<uint32_t *>(area) + wv * 256;
  if ((int)wv < nch) {
    const int k = (int)wv;
    persist_child<DT, HASV>(c, P, coff[k], clen[k], child_depth(s.depth, cdepth, s.len, clen[k], s.dmax),
                            s.dmax, s.req, out_s, cown[k], clook[k], hist);
  }
  __syncthreads();
  if (tid == 0) {
    const unsigned long long fin = (unsigned long long)band_now + P.final_keys;
    if (fin) atomicSub(&c.p.ctl[kQLeft], fin);
  }
}

// A partition task.
template <int DT, bool HASV, bool WIDE, bool DBG>
__device__ void persist_part(const Ctx &c, PersistCtl &P, unsigned char *area, const Task &t) {
  const uint32_t tid = threadIdx.x;
  TPart *tp = c.p.parts + t.id;
  const uint32_t flags = tp->s.flags;
  unsigned long long *ctr = c.p.pctr + (size_t)t.id * kCtrStride;
  if (flags & kSegTwo) {
    auto &L = *reinterpret_cast<PartLds<DT, HASV, true, kPNT> *>(area);
    partition_chunks<DT, HASV, WIDE, true, kPNT, 0, DBG>(c, (const Seg *)&tp->s, ctr, 1u, t.c0, t.c1, L);
  } else {
    auto &L = *reinterpret_cast<PartLds<DT, HASV, false, kPNT> *>(area);
    partition_chunks<DT, HASV, WIDE, false, kPNT, 0, DBG>(c, (const Seg *)&tp->s, ctr, 1u, t.c0, t.c1, L);
  }
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const uint32_t k = t.c1 - t.c0;
    const uint32_t old = atomicAdd(&tp->done, k);
    P.last = (old + k == tp->nchunks) ? 1u : 0u;
  }
  __syncthreads();
  if (!P.last) return;
  __threadfence();
  persist_plan<DT, HASV, DBG>(c, P, area, t.id);
}

// A select task: histogram of the current digit over its chunks.
template <int DT, bool HASV>
__device__ void persist_select(const Ctx &c, PersistCtl &P, unsigned char *area, const Task &t) {
  using B = typename Codec<DT>::B;
  constexpr uint32_t BITS = (uint32_t)sizeof(B) * 8;
  const uint32_t tid = threadIdx.x, wv = tid >> 6, lane = tid & 63u;
  TPart *tp = c.p.parts + t.id;
  const Seg s = tp->s;
  const uint32_t round = tp->round;
  const B prefix = (B)tp->prefix, mask = (B)tp->mask;
  const uint32_t shift = BITS - 8 * (round + 1);
  uint32_t *lh = reinterpret_cast<uint32_t *>(area);
  lh[tid] = 0u;
  __syncthreads();
  const B *Y = (const B *)((s.flags & kSegInS) ? c.S : c.K);
  constexpr int PER = (int)(kSelChunk / kPNT);   // keys per thread per chunk, loaded together
  for (uint32_t ch = t.c0; ch < t.c1; ch++) {
    const uint64_t base = (uint64_t)ch * kSelChunk + tid;
    B v[PER];
#pragma unroll
    for (int j = 0; j < PER; j++) {
      const uint64_t x = base + (uint64_t)j * kPNT;
      v[j] = x < s.len ? Y[s.off + x] : (B)0;
    }
#pragma unroll
    for (int j = 0; j < PER; j++) {
      const B u = Codec<DT>::enc(v[j]);
      if (base + (uint64_t)j * kPNT < s.len && (u & mask) == prefix)
        atomicAdd(&lh[(uint32_t)(u >> shift) & 255u], 1u);
    }
  }
  __syncthreads();
  uint32_t *gh = c.p.hist + (size_t)tp->hslot * 256;
  if (lh[tid]) atomicAdd(&gh[tid], lh[tid]);
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const uint32_t k = t.c1 - t.c0;
    const uint32_t old = atomicAdd(&tp->done, k);
    P.last = (old + k == tp->nchunks) ? 1u : 0u;
  }
  __syncthreads();
  if (!P.last || wv != 0) return;
  __threadfence();
  // the digit holding rank krem among the keys that match the prefix
  uint32_t h[4], sum = 0;
  for (int i = 0; i < 4; i++) {
    h[i] = __hip_atomic_load(&gh[lane * 4 + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sum += h[i];
  }
  const uint32_t krem = tp->krem;
  const uint32_t incl = wave_incl_scan(sum), excl = incl - sum;
  const bool mine = excl <= krem && krem < incl;
  const unsigned long long bm = __ballot(mine);
  const int src = bm ? (int)__builtin_ctzll(bm) : 63;
  uint32_t dig = lane * 4 + 3, below = excl;
  {
    uint32_t acc = excl;
    for (int i = 0; i < 4; i++) {
      if (krem < acc + h[i]) { dig = lane * 4 + i; below = acc; break; }
      acc += h[i];
    }
  }
  dig = shfl_u32(dig, src);
  below = shfl_u32(below, src);
  for (int i = 0; i < 4; i++) gh[lane * 4 + i] = 0u;
  const B np = prefix | ((B)dig << shift), nm = mask | ((B)255 << shift);
  if (lane == 0) stat_add(c, kStSelRounds, 1ull);
  if (round + 1 < BITS / 8) {
    if (lane == 0) {
      tp->round = round + 1;
      tp->prefix = (uint64_t)np;
      tp->mask = (uint64_t)nm;
      tp->krem = krem - below;
      tp->done = 0;
    }
    pool_tasks(c, t.id, kTaskSelect, tp->nchunks);
    return;
  }
  // all digits fixed: np is the exact pivot; the children's pivots from the
  // sample; a one-level partition
  uint32_t S = c.samples;
  if (S > s.len) S = (s.len & 1) ? s.len : s.len - 1;
  uint64_t piv[7];
  wave_part_pivots<DT>(Y, s.off, s.len, S, c.jitter, true, np, piv);
  const uint32_t flags = s.flags & ~(kSegSel | kSegTwo);
  const uint32_t nch = pool_chunks<DT, HASV>(c, s.off, s.len, flags);
  if (lane == 0) {
    for (int q = 0; q < 7; q++) tp->s.piv[q] = piv[q];
    tp->s.flags = flags;
    tp->s.nlt = 0;
    tp->s.neq = 0;
    tp->nchunks = nch;
    tp->done = 0;
  }
  if (lane < (uint32_t)kCtrStride) c.p.pctr[(size_t)t.id * kCtrStride + lane] = 0ull;
  pool_tasks(c, t.id, kTaskPart, nch);
}

// The persistent kernel.
template <int DT, bool HASV, bool WIDE, bool DBG = false>
__global__ __launch_bounds__(kPNT) void k_persist(Ctx c) {
  extern __shared__ __align__(16) unsigned char smem[];
  PersistCtl &P = *reinterpret_cast<PersistCtl *>(smem);
  unsigned char *area = smem + kPCtlBytes;
  const uint32_t tid = threadIdx.x;
  unsigned long long iters = 0;
  for (;;) {
    if (tid == 0) {
      uint32_t st = 0;
      const unsigned long long idx = atomicAdd(&c.p.ctl[kQHead], 1ull);
      const size_t slot = (size_t)(idx & c.p.qmask);
      for (;;) {
        if (++iters > c.p.iter_cap) { persist_abort(c, kErrIter); st = 2; break; }
        if (__hip_atomic_load(&c.p.seq[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == idx + 1) {
          P.task = c.p.task[slot];
          break;
        }
        if (__hip_atomic_load(&c.p.ctl[kQAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { st = 2; break; }
        if (__hip_atomic_load(&c.p.ctl[kQLeft], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) { st = 1; break; }
        __builtin_amdgcn_s_sleep(8);
      }
      P.state = st;
    }
    __syncthreads();
    if (P.state != 0) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const Task t = P.task;
    if (t.kind == kTaskPart) {
      persist_part<DT, HASV, WIDE, DBG>(c, P, area, t);
    } else if (t.kind == kTaskSelect) {
      persist_select<DT, HASV>(c, P, area, t);
    } else {
      const FinItem b = c.p.bands[t.id];
      FinItem it = b;
      const uint64_t at = (uint64_t)t.c0 * kBandChunk;
      it.off = b.off + at;
      it.src = b.src + at;
      it.len = b.len - (uint32_t)at < kBandChunk ? b.len - (uint32_t)at : kBandChunk;
      fill_band<DT, HASV, DBG>(c, it, tid, kPNT);
      __syncthreads();
      if (tid == 0) atomicSub(&c.p.ctl[kQLeft], (unsigned long long)it.len);
    }
    __syncthreads();
  }
}

}  // namespace tsqs
