// tsqs_dt.hip -- the launch schedule of one key type (compiled once per type
// with TSQS_DT = 0..4; see tsqs_host.hpp).
//
// One call = one schedule enqueued on the caller's stream, with no host
// synchronisation:
//   k_reset, [upload of batch offsets], [presortedness check], k_init (roots:
//   pivots or small items), then per level d: k_partition(d), k_plan(d),
//   k_finish(d) for the number of levels a median split needs
//   (ceil(log2(n / small_max)) + 2, two levels per pass after the first),
//   then k_seed + k_persist: the persistent kernel finishes whatever is left
//   (nothing, for most inputs: its workgroups see no keys left and return).
// With the persistent schedule (TSQS_OPT_SCHEDULE 1) no level is launched:
// k_finish of the roots' small arrays, then every part in k_persist.
#include "tsqs_host.hpp"
#include "tsqs_queue_state.hpp"

#include <atomic>
#include <cstring>

#ifndef TSQS_DT
#error "compile with -DTSQS_DT=<key type 0..4>"
#endif

namespace tsqs {
namespace host {
namespace {

// Workgroups of the two-level partition instance when TSQS_OPT_PART_GRID is 0.
// For 4-byte elements (keys without payload), as many as are resident at once
// (the occupancy of this instance, 7 per CU): each workgroup owns a fixed run of
// chunks, so a second round of workgroups would finish after the first, and the
// pass is latency-bound enough that every resident workgroup pays (2^28 int32,
// passes in all: 4.9 ms at 7 per CU, 5.05 at 5, 5.2 at 4; a grid one round
// larger than fits left a straggler round).  Wider elements move twice the bytes
// per chunk and keep 4 per CU (2^28 int64: passes 8.94 ms at 4, 9.06 at 5).
template <int DT, bool HASV, bool WIDE, int WGX>
int resident_grid(int cus) {
  if (HASV || sizeof(typename Codec<DT>::B) > 4) return 4 * cus;
  static std::atomic<int> per_cu{0};
  int nb = per_cu.load(std::memory_order_relaxed);
  if (nb == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_partition<DT, HASV, WIDE, true, WGX>,
                                                     WGX * kPartNT2, 0) != hipSuccess || nb < 1)
      nb = 4;
    per_cu.store(nb, std::memory_order_relaxed);
  }
  return nb * cus;
}

// The partition kernels of level d: the one-level kernel, then (d > 0 or
// `two`) the two-level kernel, each at the workgroup size the options choose
// (TSQS_OPT_PART_THREADS1 / 2: the default, or twice the threads with half the
// keys each).  grid: the one-level kernel's workgroups, and the two-level
// kernel's when TSQS_OPT_PART_GRID sets them; cus: compute units.
template <int DT, bool HASV, bool WIDE>
void launch_pass(const Ctx &c, int d, bool two, int grid, int cus, hipStream_t s) {
  const bool fixed = g_opt.part_grid > 0;
  if (c.dbg) {
    // debug shadows: the checking instances, at the default workgroup sizes
    hipLaunchKernelGGL((k_partition<DT, HASV, WIDE, false, 1, true>), dim3(grid), dim3(kPartNT1), 0, s, c, d);
    if (two)
      hipLaunchKernelGGL((k_partition<DT, HASV, WIDE, true, 1, true>), dim3(grid), dim3(kPartNT2), 0, s, c, d);
    return;
  }
  if (g_opt.part_threads1 == 2 * kPartNT1)
    hipLaunchKernelGGL((k_partition<DT, HASV, WIDE, false, 2>), dim3(grid), dim3(2 * kPartNT1), 0, s, c, d);
  else
    hipLaunchKernelGGL((k_partition<DT, HASV, WIDE, false, 1>), dim3(grid), dim3(kPartNT1), 0, s, c, d);
  if (!two) return;
  if (g_opt.part_threads2 == 2 * kPartNT2) {
    const int g2 = fixed ? grid : resident_grid<DT, HASV, WIDE, 2>(cus);
    hipLaunchKernelGGL((k_partition<DT, HASV, WIDE, true, 2>), dim3(g2), dim3(2 * kPartNT2), 0, s, c, d);
  } else {
    const int g2 = fixed ? grid : resident_grid<DT, HASV, WIDE, 1>(cus);
    hipLaunchKernelGGL((k_partition<DT, HASV, WIDE, true, 1>), dim3(g2), dim3(kPartNT2), 0, s, c, d);
  }
}

template <int DT, bool HASV>
int launch_finish(const Ctx &c, int d, int grid, size_t lds, hipStream_t s) {
  if (c.dbg)   // debug shadows: the checking instance of the default algorithm
    hipLaunchKernelGGL((k_finish<DT, HASV, 3, true>), dim3(grid), dim3(kFinNT), lds, s, c, d);
  else if (g_opt.finish_algo == 0)
    hipLaunchKernelGGL((k_finish<DT, HASV, 0>), dim3(grid), dim3(kFinNT), lds, s, c, d);
  else if (g_opt.finish_algo == 1)
    hipLaunchKernelGGL((k_finish<DT, HASV, 1>), dim3(grid), dim3(kFinNT), lds, s, c, d);
  else if (g_opt.finish_algo == 2)
    hipLaunchKernelGGL((k_finish<DT, HASV, 2>), dim3(grid), dim3(kFinNT), lds, s, c, d);
  else
    hipLaunchKernelGGL((k_finish<DT, HASV, 3>), dim3(grid), dim3(kFinNT), lds, s, c, d);
  return hipGetLastError() == hipSuccess ? TSQS_OK : TSQS_EDEVICE;
}

// Workgroups of the persistent kernel: as many as fit on the device at once
// (it needs no more, and no co-residency).
template <int DT, bool HASV, bool WIDE, bool DBG>
int persist_grid(int cus, size_t lds) {
  static int per_cu = -1;
  static size_t per_cu_lds = 0;
  if (per_cu < 0 || per_cu_lds != lds) {
    if (lds > 65536 && hipFuncSetAttribute((const void *)k_persist<DT, HASV, WIDE, DBG>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds) != hipSuccess)
      return -1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<DT, HASV, WIDE, DBG>, kPNT, lds) != hipSuccess)
      return -1;
    per_cu = nb > 0 ? nb : 1;
    per_cu_lds = lds;
  }
  return per_cu * cus;
}

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
  if (h_offs && !a.offs_ready)
    HIPCHK(hipMemcpyAsync(w.offs, h_offs, (nroots + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
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
  // debug shadows: every key takes the passes (no presortedness check), and
  // every store is checked against the shadows
  c.dbg = w.dbg;
  c.pre = (g_opt.presort && !c.dbg && !h_offs && n > small_max)
              ? (unsigned int *)(w.stats + kStripes * kStatWords + 8) : nullptr;
  c.roots = h_offs ? w.offs : nullptr;
  c.root_recs = nullptr;
  c.req_left = nullptr;
  c.req_flag = nullptr;
  c.done_ring = nullptr;
  c.done_pos = nullptr;
  c.done_cap = 0;
  c.fin_roots_only = 0;
  c.p = PCtx();
  c.root_level = 0;
  c.ring = 0;
  c.n = n;
  c.nroots = (uint32_t)nroots;
  c.small_max = small_max;
  c.wave_max = wave_max;
  c.presort_roots = (g_opt.presort && !c.dbg && h_offs) ? 1u : 0u;   // batches: each array by its wave
  c.samples = (uint32_t)g_opt.samples;
  c.depth_factor = (uint32_t)g_opt.depth_factor;
  c.pivot_mode = (uint32_t)g_opt.pivot_mode;
  c.jitter = mix32((uint64_t)g_opt.seed + (g_calls++));
  c.seg_cap = (uint32_t)seg_cap;
  c.big_cap = (uint32_t)big_cap;
  c.fin_roots_only = 0;
  // 32-bit byte offsets within a part suffice unless a part reaches 4 GiB
  const bool wide = (uint64_t)max_root * sizeof(typename Codec<DT>::B) > 0xFFFFFFFFull;
  const size_t plds = persist_lds<DT, HASV>();
  const int pgrid = c.dbg ? (wide ? persist_grid<DT, HASV, true, true>(env.cus, plds)
                                  : persist_grid<DT, HASV, false, true>(env.cus, plds))
                          : (wide ? persist_grid<DT, HASV, true, false>(env.cus, plds)
                                  : persist_grid<DT, HASV, false, false>(env.cus, plds));
  if (pgrid <= 0) return TSQS_EDEVICE;
  c.p.task = w.task; c.p.seq = w.seq; c.p.ctl = w.ctl;
  c.p.parts = w.parts; c.p.pctr = w.pctr; c.p.hist = w.hist; c.p.bands = w.bands;
  c.p.sfin = w.sfin;
  c.p.sfin_cap = (uint32_t)w.sfin_cap;
  c.p.pad2 = 0;
  c.p.qmask = (unsigned long long)w.qcap - 1;
  c.p.part_cap = (uint32_t)w.part_cap;
  c.p.hist_cap = (uint32_t)w.hist_cap;
  c.p.band_cap = (uint32_t)w.band_cap;
  c.p.grid = (uint32_t)pgrid;
  c.p.iter_cap = g_opt.iter_cap > 0 ? (unsigned long long)g_opt.iter_cap : kDefaultIterCap;

  const int part_grid = g_opt.part_grid > 0 ? (int)g_opt.part_grid : 4 * env.cus;
  const int fin_grid = g_opt.finish_grid > 0 ? (int)g_opt.finish_grid : kFinGridPerCu * env.cus;
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
    HIPCHK(hipFuncSetAttribute((const void *)k_finish_list<DT, HASV, 0>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish_list<DT, HASV, 1>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish_list<DT, HASV, 2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
    HIPCHK(hipFuncSetAttribute((const void *)k_finish_list<DT, HASV, 3>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
    if (c.dbg) {
      HIPCHK(hipFuncSetAttribute((const void *)k_finish<DT, HASV, 3, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
      HIPCHK(hipFuncSetAttribute((const void *)k_finish_list<DT, HASV, 3, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds));
    }
  }
  const size_t waves_init = (nroots + kPlanNW - 1) / kPlanNW;
  int init_grid = (int)(waves_init < (size_t)(4 * env.cus) ? waves_init : (size_t)(4 * env.cus));
  if (init_grid < 1) init_grid = 1;

  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, c);
  if (c.dbg) hipLaunchKernelGGL(k_dbg_clear, dim3(4 * env.cus), dim3(256), 0, s, c);
  if (c.dbg && g_opt.debug >= 2) hipLaunchKernelGGL(k_dbg_plant, dim3(1), dim3(64), 0, s, c, (int)g_opt.debug);
  if (c.pre) {
    const uint64_t pre_chunks = (n + (uint64_t)kPreNT * kPreRows - 1) / ((uint64_t)kPreNT * kPreRows);
    const int scan_grid = (int)(pre_chunks < (uint64_t)(8 * env.cus) ? pre_chunks : (uint64_t)(8 * env.cus));
    hipLaunchKernelGGL((k_presort_scan<DT>), dim3(scan_grid), dim3(kPreNT), 0, s, c);
    hipLaunchKernelGGL((k_presort_reverse<DT, HASV>), dim3(8 * env.cus), dim3(kPreNT), 0, s, c);
  }
  hipLaunchKernelGGL((k_init<DT, HASV>), dim3(init_grid), dim3(kPlanNT), 0, s, c);
  HIPCHK(hipGetLastError());

  // median-of-63 splits stay within about 45/55: launch the levels for 20% more
  // halvings than a perfect split, plus two (the first pass is one level, the
  // rest two levels each); every root small: level 0 has only its finish work.
  // Whatever is left after them (bad pivots, the depth limit) the persistent
  // kernel finishes, so the call never waits for the device.
  const uint32_t lv = ceil_log2((max_root + small_max - 1) / small_max);
  const bool roots_small = max_root <= small_max;
  const uint32_t lv_all = lv + (lv + 4) / 5 + 2;
  const bool persistent = g_opt.schedule == 1;
  uint32_t expected = roots_small ? 1u : 2 + lv_all / 2;
  if (persistent) expected = 0;
  if (expected > (uint32_t)kMaxLevels - 2) expected = (uint32_t)kMaxLevels - 2;
  for (int d = 0; d < (int)expected; d++) {
    const bool idle = d == 0 && roots_small;
    if (timing) HIPCHK(hipEventRecord(env.ev[2 * d], s));
    if (idle) {
    } else if (wide) {
      launch_pass<DT, HASV, true>(c, d, d > 0, part_grid, env.cus, s);
    } else {
      launch_pass<DT, HASV, false>(c, d, d > 0, part_grid, env.cus, s);
    }
    if (timing) HIPCHK(hipEventRecord(env.ev[2 * d + 1], s));
    if (!idle) hipLaunchKernelGGL((k_plan<DT, HASV>), dim3(plan_grid), dim3(kPlanNT), 0, s, c, d);
    if (launch_finish<DT, HASV>(c, d, fin_grid, fin_lds, s) != TSQS_OK) return TSQS_EDEVICE;
  }
  if (persistent) {
    // the roots' small arrays, then every part in the persistent kernel
    Ctx cr = c;
    cr.fin_roots_only = 1u;
    if (launch_finish<DT, HASV>(cr, 0, fin_grid, fin_lds, s) != TSQS_OK) return TSQS_EDEVICE;
  }
  const int seed_grid = 4 * env.cus;
  hipLaunchKernelGGL((k_seed<DT, HASV>), dim3(seed_grid), dim3(kPlanNT), 0, s, c, (int)expected);
  if (c.dbg && wide)
    hipLaunchKernelGGL((k_persist<DT, HASV, true, true>), dim3(c.p.grid), dim3(kPNT), plds, s, c);
  else if (c.dbg)
    hipLaunchKernelGGL((k_persist<DT, HASV, false, true>), dim3(c.p.grid), dim3(kPNT), plds, s, c);
  else if (wide)
    hipLaunchKernelGGL((k_persist<DT, HASV, true>), dim3(c.p.grid), dim3(kPNT), plds, s, c);
  else
    hipLaunchKernelGGL((k_persist<DT, HASV, false>), dim3(c.p.grid), dim3(kPNT), plds, s, c);
  HIPCHK(hipGetLastError());
  // the small parts the persistent kernel listed
  if (c.dbg)
    hipLaunchKernelGGL((k_finish_list<DT, HASV, 3, true>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c);
  else if (g_opt.finish_algo == 0)
    hipLaunchKernelGGL((k_finish_list<DT, HASV, 0>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c);
  else if (g_opt.finish_algo == 1)
    hipLaunchKernelGGL((k_finish_list<DT, HASV, 1>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c);
  else if (g_opt.finish_algo == 2)
    hipLaunchKernelGGL((k_finish_list<DT, HASV, 2>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c);
  else
    hipLaunchKernelGGL((k_finish_list<DT, HASV, 3>), dim3(fin_grid), dim3(kFinNT), fin_lds, s, c);
  if (c.dbg) hipLaunchKernelGGL(k_dbg_end, dim3(4 * env.cus), dim3(256), 0, s, c);
  HIPCHK(hipGetLastError());
  if (env.done) HIPCHK(hipEventRecord(env.done, s));

  LastCall &lc = g_last;
  lc.valid = true;
  lc.done = env.done;
  lc.s = s;
  lc.d_lvl = w.lvl;
  lc.d_stats = w.stats;
  lc.h_lvl = env.h_lvl;
  lc.h_stats = env.h_stats;
  lc.ev = timing ? env.ev : nullptr;
  lc.levels = expected;
  lc.roots_small = roots_small;
  lc.n = n;
  lc.kb = (uint32_t)kb;
  lc.vb = HASV ? 4u : 0u;
  lc.schedule = persistent ? 1u : 0u;
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
  c.fin_roots_only = 0;
  c.p = PCtx();
  c.dbg = nullptr;
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
  if ((uint64_t)G.max_n * G.kb > 0xFFFFFFFFull) launch_pass<DT, false, true>(c, d, true, grid, q->cus, G.s);
  else launch_pass<DT, false, false>(c, d, true, grid, q->cus, G.s);
  hipLaunchKernelGGL((k_plan<DT, false>), dim3(grid), dim3(kPlanNT), 0, G.s, c, d);
  const int fgrid = g_opt.finish_grid > 0 ? (int)g_opt.finish_grid : kFinGridPerCu * q->cus;
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
