// tsqs_dt.hip -- the launch schedule of one key type (compiled once per type
// with TSQS_DT = 0..4; see tsqs_host.hpp).
//
// One call = one schedule on the caller's stream:
//   k_reset, [upload of batch offsets], [presortedness check], k_init (roots:
//   pivots or small items), then per level d: k_partition(d), k_plan(d),
//   k_finish(d),
// launched without host synchronisation for the number of levels a median
// split needs (ceil(log2(n / small_max)) + 2, two levels per pass after the
// first); the stream is then synchronised once, and only if parts remain (bad
// pivots, the depth-limit path) more levels are launched, eight at a time.
#include "tsqs_host.hpp"
#include "tsqs_queue_state.hpp"

#include <cstring>

#ifndef TSQS_DT
#error "compile with -DTSQS_DT=<key type 0..4>"
#endif

namespace tsqs {
namespace host {
namespace {

template <int DT, bool HASV>
int run_t(const CallEnv &env, const CallArgs &a) {
  using B = typename Codec<DT>::B;
  const size_t kb = sizeof(B);
  void *keys = a.keys;
  uint32_t *vals = HASV ? a.vals : nullptr;
  const uint64_t *h_offs = a.h_offs;
  const size_t nroots = a.nroots;
  const uint64_t n = a.n, max_root = a.max_root;
  hipStream_t s = a.s;
  const WsView &w = env.v;
  if (((uintptr_t)keys % kb) != 0 || ((uintptr_t)vals % 4) != 0) return TSQS_EINVAL;
  const FinGeom geo = fin_geom<DT, HASV>(env.lds_budget, g_opt.small_max);
  const uint32_t small_max = geo.small_max, wave_max = geo.wave_max;
  const size_t seg_cap = w.seg_cap, big_cap = w.big_cap;
  if (h_offs) HIPCHK(hipMemcpyAsync(w.offs, h_offs, (nroots + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  const bool timing = g_opt.timing && env.ev;

  Ctx c;
  c.K = keys; c.S = w.S;
  c.V = vals; c.VS = w.VS; c.VE = w.VE;
  c.seg0 = w.seg[0]; c.seg1 = w.seg[1];
  c.ctr0 = w.ctr[0]; c.ctr1 = w.ctr[1];
  c.fin = w.fin; c.finw = w.finw; c.band = w.band; c.big = w.big; c.lvl = w.lvl;
  c.stats = w.stats;
  c.err = (unsigned int *)(w.stats + kStripes * kStatWords);
  // the presortedness check of a single array that needs a pass
  c.pre = (g_opt.presort && !h_offs && n > small_max)
              ? (unsigned int *)(w.stats + kStripes * kStatWords + 8) : nullptr;
  c.roots = h_offs ? w.offs : nullptr;
  c.root_recs = nullptr;
  c.req_left = nullptr;
  c.req_flag = nullptr;
  c.done_ring = nullptr;
  c.done_pos = nullptr;
  c.done_cap = 0;
  c.pad1 = 0;
  c.root_level = 0;
  c.ring = 0;
  c.n = n;
  c.nroots = (uint32_t)nroots;
  c.small_max = small_max;
  c.wave_max = wave_max;
  c.presort_roots = (g_opt.presort && h_offs) ? 1u : 0u;   // batches: each array by its wave
  c.samples = (uint32_t)g_opt.samples;
  c.depth_factor = (uint32_t)g_opt.depth_factor;
  c.pivot_mode = (uint32_t)g_opt.pivot_mode;
  c.jitter = mix32((uint64_t)g_opt.seed + (g_calls++));
  c.seg_cap = (uint32_t)seg_cap;
  c.big_cap = (uint32_t)big_cap;

  const int part_grid = g_opt.part_grid > 0 ? (int)g_opt.part_grid : 4 * env.cus;
  const int fin_grid = g_opt.finish_grid > 0 ? (int)g_opt.finish_grid : 8 * env.cus;
  const int plan_grid = 4 * env.cus;
  const size_t fin_lds = geo.fin_lds;
  if (fin_lds > 65536) {
    HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, HASV, 0>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, HASV, 1>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, HASV, 2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, HASV, 3>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
  }
  const size_t waves_init = (nroots + kPlanNW - 1) / kPlanNW;
  int init_grid = (int)(waves_init < (size_t)(4 * env.cus) ? waves_init : (size_t)(4 * env.cus));
  if (init_grid < 1) init_grid = 1;

  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, c);
  if (c.pre) {
    const uint64_t pre_chunks = (n + (uint64_t)kPreNT * kPreRows - 1) / ((uint64_t)kPreNT * kPreRows);
    const int scan_grid = (int)(pre_chunks < (uint64_t)(8 * env.cus) ? pre_chunks : (uint64_t)(8 * env.cus));
    hipLaunchKernelGGL((k_presort_scan<DT>), dim3(scan_grid), dim3(kPreNT), 0, s, c);
    hipLaunchKernelGGL((k_presort_reverse<DT, HASV>), dim3(8 * env.cus), dim3(kPreNT), 0, s, c);
  }
  hipLaunchKernelGGL((k_init<DT, HASV>), dim3(init_grid), dim3(kPlanNT), 0, s, c);
  HIPCHK(hipGetLastError());

  // median-of-63 splits stay within about 45/55: allow 20% more levels than a
  // perfect halving, plus two
  // 32-bit byte offsets within a part suffice unless a part reaches 4 GiB
  const bool wide = (uint64_t)max_root * sizeof(typename Codec<DT>::B) > 0xFFFFFFFFull;
  const uint32_t lv = ceil_log2((max_root + small_max - 1) / small_max);
  // every root small: level 0 has no parts, only its finish work.  The first
  // pass is one level and the rest two levels each (with payloads too).
  const bool roots_small = max_root <= small_max;
  const uint32_t lv_all = lv + (lv + 4) / 5 + 2;
  uint32_t expected = roots_small ? 1u : 2 + lv_all / 2;
  int d = 0, target = (int)expected;
  if (c.pre && n >= kPresortSyncMin) {
    // a large array found in order needs none of the levels: read the two words
    // of the check once instead of launching the whole schedule empty
    unsigned int *hp = (unsigned int *)(env.h_stats + kStripes * kStatWords + 8);
    HIPCHK(hipMemcpyAsync(hp, c.pre, 2 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hp[0] != 0u && hp[1] == 0u) target = 0;
  }
  if (target > kMaxLevels - 1) target = kMaxLevels - 1;
  for (;;) {
    for (; d < target; d++) {
      const bool idle = d == 0 && roots_small;
      if (timing) HIPCHK(hipEventRecord(env.ev[2 * d], s));
      if (idle) {
      } else if (wide) {
        hipLaunchKernelGGL((k_partition<DT, HASV, true, false>), dim3(part_grid), dim3(kPartNT1), 0, s, c, d);
        if (d > 0)
          hipLaunchKernelGGL((k_partition<DT, HASV, true, true>), dim3(part_grid), dim3(kPartNT2), 0, s, c, d);
      } else {
        hipLaunchKernelGGL((k_partition<DT, HASV, false, false>), dim3(part_grid), dim3(kPartNT1), 0, s, c, d);
        if (d > 0)
          hipLaunchKernelGGL((k_partition<DT, HASV, false, true>), dim3(part_grid), dim3(kPartNT2), 0, s, c, d);
      }
      if (timing) HIPCHK(hipEventRecord(env.ev[2 * d + 1], s));
      if (!idle) hipLaunchKernelGGL((k_plan<DT, HASV>), dim3(plan_grid), dim3(kPlanNT), 0, s, c, d);
      if (g_opt.finish_algo == 0)
        hipLaunchKernelGGL((k_finish<DT, HASV, 0>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c, d);
      else if (g_opt.finish_algo == 1)
        hipLaunchKernelGGL((k_finish<DT, HASV, 1>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c, d);
      else if (g_opt.finish_algo == 2)
        hipLaunchKernelGGL((k_finish<DT, HASV, 2>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c, d);
      else
        hipLaunchKernelGGL((k_finish<DT, HASV, 3>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c, d);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(env.h_lvl, w.lvl, sizeof(LevelCtl) * (size_t)(d + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(env.h_stats, w.stats, sizeof(unsigned long long) * (kStripes * kStatWords + 1),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*(unsigned int *)(env.h_stats + kStripes * kStatWords)) return TSQS_EINTERNAL;
    if ((env.h_lvl[d].packed >> 40) == 0) break;
    if (d >= kMaxLevels - 1) return TSQS_EINTERNAL;
    target = d + 8 < kMaxLevels - 1 ? d + 8 : kMaxLevels - 1;
  }

  tsqs_stats_t &st = g_stats;
  std::memset(&st, 0, sizeof st);
  st.levels = (uint32_t)d;
  st.n = n;
  st.key_bytes = (uint32_t)kb;
  st.payload_bytes = HASV ? 4u : 0u;
  for (int i = 0; i < kStripes; i++) {
    const unsigned long long *sp = env.h_stats + (size_t)i * kStatWords;
    st.fallback_parts += sp[kStFallback];
    st.small_parts += sp[kStSmallParts];
    st.small_keys += sp[kStSmallKeys];
    st.band_keys += sp[kStBandKeys];
    st.presorted += (uint32_t)(sp[kStPresorted] + sp[kStPresortedRoots]);
  }
  for (int i = 0; i < d; i++)
    if (env.h_lvl[i].packed >> 40) st.max_depth = (uint32_t)i;
  for (int i = 0; i < d && i < TSQS_MAX_LEVELS; i++) {
    st.level_keys[i] = env.h_lvl[i].keys;
    st.level_parts[i] = (uint32_t)(env.h_lvl[i].packed >> 40);
    st.partition_bytes += 2ull * env.h_lvl[i].keys * (kb + (HASV ? 4 : 0));
    if (!(i == 0 && roots_small)) st.partition_launches++;
    if (timing) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, env.ev[2 * i], env.ev[2 * i + 1]));
      st.level_ms[i] = ms;
      st.partition_ms += ms;
    }
  }
  g_have_stats = true;
  return TSQS_OK;
}

}  // namespace

template <int DT>
int sort_dt(const CallEnv &env, const CallArgs &a, bool hasv) {
  return hasv ? run_t<DT, true>(env, a) : run_t<DT, false>(env, a);
}

template <int DT>
FinGeom geom_dt(size_t lds_budget, bool hasv) {
  return hasv ? fin_geom<DT, true>(lds_budget, g_opt.small_max)
              : fin_geom<DT, false>(lds_budget, g_opt.small_max);
}

template <int DT>
int queue_tick(tsqs_queue *q, QGroup &G) {
  const int slot = (int)(G.tick % kInFlight);
  if (G.ev_used[slot]) {
    const hipError_t e = hipEventQuery(G.ev[slot]);
    if (e == hipErrorNotReady) return TSQS_EAGAIN;
    if (e != hipSuccess) return TSQS_EDEVICE;
    G.ev_used[slot] = false;
    if (G.h_err[slot]) { q->broken = true; return TSQS_EINTERNAL; }
  }
  const int d = (int)(G.tick % kMaxLevels);
  const int dn = (d + 1) % kMaxLevels;
  const uint32_t nroots = (uint32_t)G.next_roots.size();
  Ctx c;
  c.K = q->KA; c.S = q->SA;
  c.V = nullptr; c.VS = nullptr; c.VE = nullptr;
  c.seg0 = G.seg[0]; c.seg1 = G.seg[1];
  c.ctr0 = G.ctr[0]; c.ctr1 = G.ctr[1];
  c.fin = G.fin; c.finw = G.finw; c.band = G.band; c.big = G.big; c.lvl = G.lvl;
  c.stats = G.stats;
  c.err = (unsigned int *)(G.stats + kStripes * kStatWords);
  c.pre = nullptr;
  c.roots = nullptr;
  c.root_recs = G.d_roots[slot];
  c.req_left = q->req_left;
  c.req_flag = q->d_flag;
  c.done_ring = q->d_ring;
  c.done_pos = q->d_pos;
  c.done_cap = kQMaxReq;
  c.pad1 = 0;
  c.root_level = d;
  c.ring = 1;
  c.n = 0;
  c.nroots = nroots;
  c.small_max = G.geo.small_max;
  c.wave_max = G.geo.wave_max;
  c.presort_roots = 0;
  c.samples = (uint32_t)g_opt.samples;
  c.depth_factor = (uint32_t)g_opt.depth_factor;
  c.pivot_mode = (uint32_t)g_opt.pivot_mode;
  c.jitter = mix32((uint64_t)g_opt.seed + 0x51ull * G.tick + (uint64_t)DT);
  c.seg_cap = (uint32_t)G.seg_cap;
  c.big_cap = (uint32_t)G.big_cap;
  if (nroots) {
    std::memcpy(G.h_roots[slot], G.next_roots.data(), sizeof(RootRec) * nroots);
    HIPCHK(hipMemcpyAsync(G.d_roots[slot], G.h_roots[slot], sizeof(RootRec) * nroots,
                          hipMemcpyHostToDevice, G.s));
  }
  const int grid = 4 * q->cus;
  hipLaunchKernelGGL(k_level_clear, dim3(1), dim3(64), 0, G.s, c, dn);
  if (nroots) {
    const uint32_t wgs = (nroots + kPlanNW - 1) / kPlanNW;
    hipLaunchKernelGGL((k_init<DT, false>), dim3(wgs < (uint32_t)grid ? wgs : (uint32_t)grid),
                       dim3(kPlanNT), 0, G.s, c);
  }
  if ((uint64_t)G.max_n * G.kb > 0xFFFFFFFFull) {
    hipLaunchKernelGGL((k_partition<DT, false, true, false>), dim3(grid), dim3(kPartNT1), 0, G.s, c, d);
    hipLaunchKernelGGL((k_partition<DT, false, true, true>), dim3(grid), dim3(kPartNT2), 0, G.s, c, d);
  } else {
    hipLaunchKernelGGL((k_partition<DT, false, false, false>), dim3(grid), dim3(kPartNT1), 0, G.s, c, d);
    hipLaunchKernelGGL((k_partition<DT, false, false, true>), dim3(grid), dim3(kPartNT2), 0, G.s, c, d);
  }
  hipLaunchKernelGGL((k_plan<DT, false>), dim3(grid), dim3(kPlanNT), 0, G.s, c, d);
  const int fgrid = g_opt.finish_grid > 0 ? (int)g_opt.finish_grid : 8 * q->cus;
  if (g_opt.finish_algo == 0)
    hipLaunchKernelGGL((k_finish<DT, false, 0>), dim3(fgrid), dim3(kFinNT), G.geo.fin_lds, G.s, c, d);
  else if (g_opt.finish_algo == 1)
    hipLaunchKernelGGL((k_finish<DT, false, 1>), dim3(fgrid), dim3(kFinNT), G.geo.fin_lds, G.s, c, d);
  else if (g_opt.finish_algo == 2)
    hipLaunchKernelGGL((k_finish<DT, false, 2>), dim3(fgrid), dim3(kFinNT), G.geo.fin_lds, G.s, c, d);
  else
    hipLaunchKernelGGL((k_finish<DT, false, 3>), dim3(fgrid), dim3(kFinNT), G.geo.fin_lds, G.s, c, d);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(&G.h_err[slot], c.err, sizeof(unsigned int), hipMemcpyDeviceToHost, G.s));
  HIPCHK(hipEventRecord(G.ev[slot], G.s));
  G.ev_used[slot] = true;
  G.next_roots.clear();
  G.tick++;
  return TSQS_OK;
}

template <int DT>
int queue_fin_lds(const FinGeom &geo) {
  if (geo.fin_lds > 65536) {
    HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, false, 0>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)geo.fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, false, 1>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)geo.fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, false, 2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)geo.fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, false, 3>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)geo.fin_lds));
  }
  return TSQS_OK;
}


template int sort_dt<TSQS_DT>(const CallEnv &, const CallArgs &, bool);
template FinGeom geom_dt<TSQS_DT>(size_t, bool);
template int queue_tick<TSQS_DT>(tsqs_queue *, QGroup &);
template int queue_fin_lds<TSQS_DT>(const FinGeom &);

}  // namespace host
}  // namespace tsqs
