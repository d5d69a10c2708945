// tsqs_host.hip -- C ABI of libtsqs (include/tsqs.h, include/tsqs_queue.h):
// argument checks, options, the per-device workspace, statistics, the records
// entry point, the autotuner and the serving queue.  The launch schedule of
// each key type is in tsqs_dt.hip.
#include "tsqs_host.hpp"
#include "tsqs_queue_state.hpp"
#include "tsqs_records.hpp"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <climits>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

namespace tsqs {
namespace host {
Options g_opt;
std::mutex g_mu;
uint64_t g_calls = 0;
LastCall g_last;
}  // namespace host
}  // namespace tsqs

using namespace tsqs;
using namespace tsqs::host;

// A captured sort (tsqs_graph_*): its own workspace, so that calls of the
// library between launches can neither reuse nor regrow the buffers the graph's
// kernels hold.
struct tsqs_graph {
  int dev = 0;
  Workspace w;
  hipStream_t cs = nullptr;        // the capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;       // recorded after each launch
  hipStream_t last = nullptr;
  bool launched = false;
  LastCall lc;                     // what its statistics read
};

namespace {

// Buffers of tsqs_sort_records per device: the index (the sorted "pointer array"),
// the staging buffer of an in-place gather, and an error word.
constexpr size_t kMaxRecBytes = 65536;
struct RecWs {
  uint32_t *idx = nullptr;
  size_t idx_cap = 0;
  unsigned char *tmp = nullptr;
  size_t tmp_cap = 0;
  unsigned int *err = nullptr;
  size_t err_cap = 0;
};
std::mutex g_rec_mu;
std::vector<RecWs> g_rec;
std::vector<Workspace> g_ws;

void free_ws(Workspace &w) {
  (void)hipFree(w.S); (void)hipFree(w.VS); (void)hipFree(w.VE);
  for (int i = 0; i < 2; i++) { (void)hipFree(w.seg[i]); (void)hipFree(w.ctr[i]); }
  (void)hipFree(w.fin); (void)hipFree(w.finw); (void)hipFree(w.band); (void)hipFree(w.big);
  (void)hipFree(w.lvl); (void)hipFree(w.stats); (void)hipFree(w.offs);
  (void)hipHostFree(w.h_lvl); (void)hipHostFree(w.h_stats);
  if (w.ev_ok) for (int i = 0; i < 2 * kMaxLevels; i++) (void)hipEventDestroy(w.ev[i]);
  (void)hipFree(w.task); (void)hipFree(w.seq); (void)hipFree(w.ctl);
  (void)hipFree(w.parts); (void)hipFree(w.pctr); (void)hipFree(w.hist); (void)hipFree(w.bands);
  (void)hipFree(w.sfin);
  (void)hipFree(w.dbg);
  if (w.done) (void)hipEventDestroy(w.done);
  w = Workspace();
}

int ensure_static(Workspace &w, int dev, hipStream_t s) {
  if (w.init) return TSQS_OK;
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  w.cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  w.lds_budget = prop.sharedMemPerBlock > 0 ? (size_t)prop.sharedMemPerBlock : 65536;
  if (hipMalloc(&w.lvl, sizeof(LevelCtl) * kMaxLevels) != hipSuccess) return TSQS_ENOMEM;
  const size_t stat_bytes = sizeof(unsigned long long) * (kStripes * kStatWords + 16);
  if (hipMalloc(&w.stats, stat_bytes) != hipSuccess) return TSQS_ENOMEM;
  if (hipHostMalloc(&w.h_lvl, sizeof(LevelCtl) * kMaxLevels, hipHostMallocDefault) != hipSuccess) return TSQS_ENOMEM;
  if (hipHostMalloc(&w.h_stats, stat_bytes, hipHostMallocDefault) != hipSuccess) return TSQS_ENOMEM;
  if (hipMalloc(&w.ctl, sizeof(unsigned long long) * kQWords) != hipSuccess) return TSQS_ENOMEM;
  HIPCHK(hipMemsetAsync(w.ctl, 0, sizeof(unsigned long long) * kQWords, s));
  HIPCHK(hipEventCreateWithFlags(&w.done, hipEventDisableTiming));
  w.init = true;
  return TSQS_OK;
}

// The workspace's buffers may be freed (grown) only after the work that uses
// them: the last call's completion.
int ws_quiesce(Workspace &w) {
  if (w.done_rec) HIPCHK(hipEventSynchronize(w.done));
  return TSQS_OK;
}

// Device bytes the workspace holds once grown to what nd needs.
size_t ws_bytes_after(const Workspace &w, const WsNeed &nd, bool hasv) {
  auto mx = [](size_t a, size_t b) { return a > b ? a : b; };
  size_t t = mx(w.s_bytes, nd.s_bytes);
  if (hasv || w.v_cap) t += 2 * mx(w.v_cap, hasv ? nd.v_elems : 0) * sizeof(uint32_t);
  const size_t seg = mx(w.seg_cap, nd.seg_cap);
  t += 2 * seg * (sizeof(Seg) + kCtrStride * sizeof(unsigned long long));
  t += 2 * mx(w.slot_cap, nd.slot_cap) * sizeof(FinItem);
  t += (mx(w.band_cap, nd.band_cap) + mx(w.big_cap, nd.big_cap)) * sizeof(FinItem);
  t += mx(w.off_cap, nd.offs) * sizeof(uint64_t);
  t += mx(w.qcap, nd.qcap) * (sizeof(Task) + sizeof(unsigned long long));
  t += mx(w.part_cap, nd.part_cap) * (sizeof(TPart) + kCtrStride * sizeof(unsigned long long));
  t += mx(w.hist_cap, nd.hist_cap) * 256 * sizeof(uint32_t);
  t += (mx(w.lband_cap, nd.lband_cap) + mx(w.sfin_cap, nd.sfin_cap)) * sizeof(FinItem);
  t += mx(w.dbg_cap, nd.dbg) * sizeof(unsigned int);
  return t;
}

// Workspace buffers of the allocating entry points, grown to what the call needs
// (TSQS_ENOMEM, with nothing allocated or freed, past TSQS_OPT_WORKSPACE_CAP).
int ws_grow(Workspace &w, const WsNeed &nd, bool hasv, WsView *v, hipStream_t s) {
  int rc;
  if (g_opt.workspace_cap > 0 && ws_bytes_after(w, nd, hasv) > (size_t)g_opt.workspace_cap)
    return TSQS_ENOMEM;
  const bool grows = w.s_bytes < nd.s_bytes || (hasv && w.v_cap < nd.v_elems) || w.seg_cap < nd.seg_cap ||
                     w.slot_cap < nd.slot_cap || w.band_cap < nd.band_cap || w.big_cap < nd.big_cap ||
                     (nd.offs && w.off_cap < nd.offs) || w.qcap < nd.qcap || w.part_cap < nd.part_cap ||
                     w.hist_cap < nd.hist_cap || w.lband_cap < nd.lband_cap || w.sfin_cap < nd.sfin_cap;
  if (grows && (rc = ws_quiesce(w)) != TSQS_OK) return rc;
  {
    size_t cap_bytes = w.s_bytes;
    void *S = w.S;
    if ((rc = grow<unsigned char>((unsigned char **)&S, &cap_bytes, nd.s_bytes)) != TSQS_OK) return rc;
    w.S = S; w.s_bytes = cap_bytes;
  }
  if (hasv) {
    size_t c1 = w.v_cap, c2 = w.v_cap;
    if ((rc = grow(&w.VS, &c1, nd.v_elems)) != TSQS_OK) return rc;
    if ((rc = grow(&w.VE, &c2, nd.v_elems)) != TSQS_OK) return rc;
    w.v_cap = c1 < c2 ? c1 : c2;
  }
  if (w.seg_cap < nd.seg_cap) {
    for (int i = 0; i < 2; i++) {
      size_t a = w.seg_cap, b = w.seg_cap * kCtrStride;
      if ((rc = grow(&w.seg[i], &a, nd.seg_cap)) != TSQS_OK) return rc;
      if ((rc = grow(&w.ctr[i], &b, nd.seg_cap * kCtrStride)) != TSQS_OK) return rc;
    }
    w.seg_cap = nd.seg_cap;
  }
  if (w.slot_cap < nd.slot_cap) {
    size_t a = w.slot_cap, b = w.slot_cap;
    if ((rc = grow(&w.fin, &a, nd.slot_cap)) != TSQS_OK) return rc;
    if ((rc = grow(&w.finw, &b, nd.slot_cap)) != TSQS_OK) return rc;
    w.slot_cap = nd.slot_cap;
  }
  if ((rc = grow(&w.band, &w.band_cap, nd.band_cap)) != TSQS_OK) return rc;
  if ((rc = grow(&w.big, &w.big_cap, nd.big_cap)) != TSQS_OK) return rc;
  if (nd.offs && (rc = grow(&w.offs, &w.off_cap, nd.offs)) != TSQS_OK) return rc;
  if (w.qcap < nd.qcap) {
    // a new ring: its sequence words and indices start from zero
    size_t a = w.qcap, b = w.qcap;
    if ((rc = grow(&w.task, &a, nd.qcap)) != TSQS_OK) return rc;
    if ((rc = grow(&w.seq, &b, nd.qcap)) != TSQS_OK) return rc;
    HIPCHK(hipMemsetAsync(w.seq, 0, sizeof(unsigned long long) * nd.qcap, s));
    HIPCHK(hipMemsetAsync(w.ctl, 0, sizeof(unsigned long long) * kQWords, s));
    w.qcap = nd.qcap;
  }
  if (w.part_cap < nd.part_cap) {
    size_t a = w.part_cap, b = w.part_cap * kCtrStride;
    if ((rc = grow(&w.parts, &a, nd.part_cap)) != TSQS_OK) return rc;
    if ((rc = grow(&w.pctr, &b, nd.part_cap * kCtrStride)) != TSQS_OK) return rc;
    w.part_cap = nd.part_cap;
  }
  if (w.hist_cap < nd.hist_cap) {
    size_t a = w.hist_cap * 256;
    if ((rc = grow(&w.hist, &a, nd.hist_cap * 256)) != TSQS_OK) return rc;
    w.hist_cap = nd.hist_cap;
  }
  if ((rc = grow(&w.bands, &w.lband_cap, nd.lband_cap)) != TSQS_OK) return rc;
  if ((rc = grow(&w.sfin, &w.sfin_cap, nd.sfin_cap)) != TSQS_OK) return rc;
  if (nd.dbg && (rc = grow(&w.dbg, &w.dbg_cap, nd.dbg)) != TSQS_OK) return rc;
  if (g_opt.timing && !w.ev_ok) {
    for (int i = 0; i < 2 * kMaxLevels; i++) HIPCHK(hipEventCreate(&w.ev[i]));
    w.ev_ok = true;
  }
  v->S = w.S; v->VS = w.VS; v->VE = w.VE;
  for (int i = 0; i < 2; i++) { v->seg[i] = w.seg[i]; v->ctr[i] = w.ctr[i]; }
  v->fin = w.fin; v->finw = w.finw; v->band = w.band; v->big = w.big;
  v->lvl = w.lvl; v->stats = w.stats; v->offs = w.offs;
  v->seg_cap = nd.seg_cap; v->slot_cap = nd.slot_cap; v->big_cap = nd.big_cap;
  v->task = w.task; v->seq = w.seq; v->ctl = w.ctl; v->parts = w.parts; v->pctr = w.pctr;
  v->hist = w.hist; v->bands = w.bands; v->sfin = w.sfin;
  v->qcap = w.qcap; v->part_cap = w.part_cap; v->hist_cap = w.hist_cap; v->band_cap = w.lband_cap;
  v->sfin_cap = w.sfin_cap;
  v->dbg = nd.dbg ? w.dbg : nullptr;
  return TSQS_OK;
}

int sort_any(int dt, const CallEnv &env, const CallArgs &a) {
  const bool hv = a.vals != nullptr;
  switch (dt) {
    case TSQS_INT32: return sort_dt<0>(env, a, hv);
    case TSQS_UINT32: return sort_dt<1>(env, a, hv);
    case TSQS_INT64: return sort_dt<2>(env, a, hv);
    case TSQS_UINT64: return sort_dt<3>(env, a, hv);
    case TSQS_FLOAT32: return sort_dt<4>(env, a, hv);
    default: return TSQS_EUNSUPPORTED;
  }
}

FinGeom geom_any(int dt, size_t lds, bool hasv) {
  switch (dt) {
    case TSQS_INT32: return geom_dt<0>(lds, hasv);
    case TSQS_UINT32: return geom_dt<1>(lds, hasv);
    case TSQS_INT64: return geom_dt<2>(lds, hasv);
    case TSQS_UINT64: return geom_dt<3>(lds, hasv);
    default: return geom_dt<4>(lds, hasv);
  }
}

// record = false: the call leaves the statistics of the caller's last call in
// place (sorts the serving queue runs for its requests).
int dispatch(void *keys, uint32_t *vals, const uint64_t *h_offs, size_t nroots, uint64_t n,
             uint64_t max_root, int dt, hipStream_t s, bool record = true) {
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0) return TSQS_EDEVICE;
  if ((size_t)dev >= g_ws.size()) g_ws.resize((size_t)dev + 1);
  Workspace &w = g_ws[(size_t)dev];
  int rc = ensure_static(w, dev, s);
  if (rc != TSQS_OK) return rc;
  const LastCall saved = g_last;
  g_last.valid = false;
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  const bool hv = vals != nullptr;
  const FinGeom geo = geom_any(dt, w.lds_budget, hv);
  WsNeed nd = ws_need(n, nroots, dt_bytes(dt), hv, geo.small_max, h_offs != nullptr);
  if (g_opt.debug) nd.dbg = 3 * (size_t)n;
  CallEnv env;
  // one workspace per device: a call on another stream starts after the last one
  if (w.done_rec && w.last_stream != s) HIPCHK(hipStreamWaitEvent(s, w.done, 0));
  if ((rc = ws_grow(w, nd, hv, &env.v, s)) != TSQS_OK) return rc;
  env.cus = w.cus;
  env.lds_budget = w.lds_budget;
  env.h_lvl = w.h_lvl;
  env.h_stats = w.h_stats;
  env.ev = w.ev_ok ? w.ev : nullptr;
  env.done = w.done;
  CallArgs a;
  a.keys = keys; a.vals = vals; a.h_offs = h_offs; a.nroots = nroots; a.n = n;
  a.max_root = max_root; a.s = s;
  rc = sort_any(dt, env, a);
  if (rc == TSQS_OK) {
    w.done_rec = true;
    w.last_stream = s;
  }
  if (!record) g_last = saved;
  return rc;
}

// Statistics of the last call (waits for its completion).
int stats_of_last(tsqs_stats_t *out) {
  const LastCall &lc = g_last;
  if (!lc.valid) return TSQS_EINVAL;
  if (lc.done) HIPCHK(hipEventSynchronize(lc.done));
  else HIPCHK(hipStreamSynchronize(lc.s));
  const size_t nlv = (size_t)lc.levels + 1;
  const size_t nst = kStripes * kStatWords + 16;
  HIPCHK(hipMemcpy(lc.h_lvl, lc.d_lvl, sizeof(LevelCtl) * nlv, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(lc.h_stats, lc.d_stats, sizeof(unsigned long long) * nst, hipMemcpyDeviceToHost));
  tsqs_stats_t &st = *out;
  std::memset(&st, 0, sizeof st);
  st.levels = lc.levels;
  st.n = lc.n;
  st.key_bytes = lc.kb;
  st.payload_bytes = lc.vb;
  st.schedule = lc.schedule;
  for (int i = 0; i < kStripes; i++) {
    const unsigned long long *sp = lc.h_stats + (size_t)i * kStatWords;
    st.fallback_parts += sp[kStFallback];
    st.small_parts += sp[kStSmallParts];
    st.small_keys += sp[kStSmallKeys];
    st.band_keys += sp[kStBandKeys];
    st.presorted += (uint32_t)(sp[kStPresorted] + sp[kStPresortedRoots]);
    st.tail_parts += sp[kStTailParts];
    st.tail_keys += sp[kStTailKeys];
    st.select_rounds += sp[kStSelRounds];
  }
  for (uint32_t i = 0; i < lc.levels; i++)
    if (lc.h_lvl[i].packed >> 40) st.max_depth = i;
  for (uint32_t i = 0; i < lc.levels && i < TSQS_MAX_LEVELS; i++) {
    st.level_keys[i] = lc.h_lvl[i].keys;
    st.level_parts[i] = (uint32_t)(lc.h_lvl[i].packed >> 40);
    st.partition_bytes += 2ull * lc.h_lvl[i].keys * (lc.kb + lc.vb);
    if (!(i == 0 && lc.roots_small)) st.partition_launches++;
    if (lc.ev) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, lc.ev[2 * i], lc.ev[2 * i + 1]));
      st.level_ms[i] = ms;
      st.partition_ms += ms;
    }
  }
  st.tail_bytes = 2ull * st.tail_keys * (lc.kb + lc.vb);
  st.error_flags = (uint32_t)lc.h_stats[kStripes * kStatWords];
  return st.error_flags ? TSQS_EINTERNAL : TSQS_OK;
}

// ---- tuning cache (TSQS_TUNE_CACHE): one text line per tuned shape ----------
//   <arch> dt=<t> v=<0|1> b=<0|1> lg=<ceil log2 n> | small_max=.. samples=..
//   part_grid=.. finish_grid=.. finish_algo=.. part_threads1=.. part_threads2=..
//   ms_default=.. ms_best=..
// The last valid line for a key wins.

std::mutex g_tune_mu;

bool tune_values_ok(const Options &o) {
  return o.small_max >= 16 && o.small_max <= 8192 && o.samples >= 3 && o.samples <= 63 &&
         (o.samples & 1) && o.part_grid >= 0 && o.part_grid <= 65536 && o.finish_grid >= 0 &&
         o.finish_grid <= 65536 && o.finish_algo >= 0 && o.finish_algo <= 3 &&
         (o.part_threads1 == kPartNT1 || o.part_threads1 == 2 * kPartNT1) &&
         (o.part_threads2 == kPartNT2 || o.part_threads2 == 2 * kPartNT2);
}

bool tune_cache_find(const char *path, const std::string &key, Options *o, double *md, double *mb) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    const char *bar = std::strstr(line, " | ");
    if (!bar || (size_t)(bar - line) != key.size() || std::strncmp(line, key.c_str(), key.size()) != 0) continue;
    Options t = *o;
    long long sm, sa, pg, fg, fa, p1, p2;
    double d0, d1;
    if (std::sscanf(bar + 3,
                    "small_max=%lld samples=%lld part_grid=%lld finish_grid=%lld finish_algo=%lld "
                    "part_threads1=%lld part_threads2=%lld ms_default=%lf ms_best=%lf",
                    &sm, &sa, &pg, &fg, &fa, &p1, &p2, &d0, &d1) != 9)
      continue;
    t.small_max = sm; t.samples = sa; t.part_grid = pg; t.finish_grid = fg; t.finish_algo = fa;
    t.part_threads1 = p1; t.part_threads2 = p2;
    if (!tune_values_ok(t)) continue;
    *o = t; *md = d0; *mb = d1;
    found = true;
  }
  std::fclose(f);
  return found;
}

void tune_cache_append(const char *path, const std::string &key, const Options &o, double md, double mb) {
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "%s | small_max=%lld samples=%lld part_grid=%lld finish_grid=%lld finish_algo=%lld "
               "part_threads1=%lld part_threads2=%lld ms_default=%.4f ms_best=%.4f\n",
               key.c_str(), (long long)o.small_max, (long long)o.samples, (long long)o.part_grid,
               (long long)o.finish_grid, (long long)o.finish_algo, (long long)o.part_threads1,
               (long long)o.part_threads2, md, mb);
  std::fclose(f);
}

// ---- autotuner inputs: seeded uniform keys (SplitMix64) and payload = index ----

__global__ void k_tune_keys(void *out, uint64_t n, int kb, uint64_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    if (kb == 4) ((uint32_t *)out)[i] = (uint32_t)z;
    else ((uint64_t *)out)[i] = z;
  }
}

__global__ void k_tune_iota(uint32_t *v, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) v[i] = (uint32_t)i;
}

}  // namespace

namespace {

// Device bytes of one group's tables for an arena of `elems` keys.
size_t group_table_bytes(size_t elems, uint32_t small_max, size_t *seg_cap, size_t *slot_cap,
                         size_t *big_cap) {
  const size_t sc = elems / ((size_t)small_max + 1) + 2;
  const size_t fc = 4 * sc + kQRootsPerTick;
  const size_t bc = 2 * (elems / kBandChunk) + 16;
  if (seg_cap) *seg_cap = sc;
  if (slot_cap) *slot_cap = fc;
  if (big_cap) *big_cap = bc;
  return 2 * sc * (sizeof(Seg) + kCtrStride * sizeof(unsigned long long)) +
         2 * fc * sizeof(FinItem) + 3 * sc * sizeof(FinItem) + bc * sizeof(FinItem) +
         sizeof(LevelCtl) * kMaxLevels + sizeof(unsigned long long) * (kStripes * kStatWords + 16) +
         kInFlight * kQRootsPerTick * sizeof(RootRec);
}

FinGeom queue_geom(int dt, size_t lds) { return geom_any(dt, lds, false); }

int group_init(tsqs_queue *q, int dt) {
  QGroup &G = q->g[dt];
  if (G.ready) return TSQS_OK;
  G.dt = dt;
  G.kb = dt_bytes(dt);
  G.geo = queue_geom(dt, q->lds_budget);
  HIPCHK(hipStreamCreateWithFlags(&G.s, hipStreamNonBlocking));
  const size_t elems = q->arena_bytes / G.kb;
  group_table_bytes(elems, G.geo.small_max, &G.seg_cap, &G.slot_cap, &G.big_cap);
  size_t c0 = 0;
  for (int i = 0; i < 2; i++) {
    c0 = 0; if (grow(&G.seg[i], &c0, G.seg_cap) != TSQS_OK) return TSQS_ENOMEM;
    c0 = 0; if (grow(&G.ctr[i], &c0, G.seg_cap * kCtrStride) != TSQS_OK) return TSQS_ENOMEM;
  }
  c0 = 0; if (grow(&G.fin, &c0, G.slot_cap) != TSQS_OK) return TSQS_ENOMEM;
  c0 = 0; if (grow(&G.finw, &c0, G.slot_cap) != TSQS_OK) return TSQS_ENOMEM;
  c0 = 0; if (grow(&G.band, &c0, 3 * G.seg_cap) != TSQS_OK) return TSQS_ENOMEM;
  c0 = 0; if (grow(&G.big, &c0, G.big_cap) != TSQS_OK) return TSQS_ENOMEM;
  c0 = 0; if (grow(&G.lvl, &c0, (size_t)kMaxLevels) != TSQS_OK) return TSQS_ENOMEM;
  c0 = 0; if (grow(&G.stats, &c0, (size_t)(kStripes * kStatWords + 16)) != TSQS_OK) return TSQS_ENOMEM;
  HIPCHK(hipMemsetAsync(G.lvl, 0, sizeof(LevelCtl) * kMaxLevels, G.s));
  HIPCHK(hipMemsetAsync(G.stats, 0, sizeof(unsigned long long) * (kStripes * kStatWords + 16), G.s));
  for (int i = 0; i < kInFlight; i++) {
    c0 = 0; if (grow(&G.d_roots[i], &c0, (size_t)kQRootsPerTick) != TSQS_OK) return TSQS_ENOMEM;
    if (hipHostMalloc(&G.h_roots[i], sizeof(RootRec) * kQRootsPerTick, hipHostMallocDefault) != hipSuccess)
      return TSQS_ENOMEM;
  }
  if (hipHostMalloc(&G.h_err, sizeof(unsigned int) * kInFlight, hipHostMallocDefault) != hipSuccess)
    return TSQS_ENOMEM;
  for (int i = 0; i < kInFlight; i++) {
    G.h_err[i] = 0;
    HIPCHK(hipEventCreateWithFlags(&G.ev[i], hipEventDisableTiming));
  }
  G.ev_made = true;
  HIPCHK(hipStreamSynchronize(G.s));
  G.ready = true;
  return TSQS_OK;
}

void group_free(QGroup &G) {
  for (int i = 0; i < 2; i++) { (void)hipFree(G.seg[i]); (void)hipFree(G.ctr[i]); }
  (void)hipFree(G.fin); (void)hipFree(G.finw); (void)hipFree(G.band); (void)hipFree(G.big);
  (void)hipFree(G.lvl); (void)hipFree(G.stats);
  for (int i = 0; i < kInFlight; i++) { (void)hipFree(G.d_roots[i]); (void)hipHostFree(G.h_roots[i]); }
  (void)hipHostFree(G.h_err);
  if (G.ev_made) for (int i = 0; i < kInFlight; i++) (void)hipEventDestroy(G.ev[i]);
  if (G.s) (void)hipStreamDestroy(G.s);
  G = QGroup();
}

// First-fit reservation of `bytes` (a multiple of kArenaAlign) in the arenas.
bool arena_take(tsqs_queue *q, uint64_t bytes, uint64_t *off) {
  for (auto it = q->free_ranges.begin(); it != q->free_ranges.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const uint64_t rest = it->second - bytes, at = it->first + bytes;
      q->free_ranges.erase(it);
      if (rest) q->free_ranges[at] = rest;
      q->arena_used += bytes;
      return true;
    }
  }
  return false;
}

void arena_give(tsqs_queue *q, uint64_t off, uint64_t bytes) {
  q->arena_used -= bytes;
  auto it = q->free_ranges.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != q->free_ranges.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    q->free_ranges.erase(nx);
  }
  if (it != q->free_ranges.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      q->free_ranges.erase(it);
    }
  }
}

// Requests the device has appended to the completion ring become done (the
// ring is read in order up to the first entry not yet written).
void collect_done(tsqs_queue *q) {
  while (!q->direct.empty()) {
    const hipError_t e = hipEventQuery(q->direct.front().second);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) { q->broken = true; break; }
    const uint64_t tk = q->direct.front().first;
    q->ev_free.push_back(q->direct.front().second);
    q->direct.pop_front();
    QReq &r = q->reqs[tk];
    r.state = 2;
    q->n_done++;
    q->reap.push_back(tk);
  }
  for (;;) {
    unsigned int *e = &q->h_ring[q->ring_cur % kQMaxReq];
    const unsigned int v = __atomic_load_n(e, __ATOMIC_ACQUIRE);
    if (v == 0) break;
    *e = 0u;
    q->ring_cur++;
    const uint64_t tk = q->id_ticket[v - 1];
    QReq &r = q->reqs[tk];
    r.state = 2;
    q->n_done++;
    q->g[r.dt].live--;
    q->reap.push_back(tk);
  }
}

// FIFO admission: copy the keys in, register the root with its group.
int admit(tsqs_queue *q) {
  while (!q->pending.empty()) {
    const uint64_t tk = q->pending.front();
    QReq &r = q->reqs[tk];
    QGroup &G = q->g[r.dt];
    if (!G.ready) {
      const int rc = group_init(q, r.dt);
      if (rc != TSQS_OK) return rc;
    }
    const bool direct = q->direct_min > 0 && r.n >= q->direct_min;
    if (direct) {
      // a large request: the single-array schedule on the queue's direct
      // stream, in place in the arena (its own launches are already efficient;
      // it does not wait for ticks), done when its event has completed
      uint64_t off = 0;
      if (!arena_take(q, r.bytes, &off)) break;
      r.boff = off;
      if (!q->ds_waits_src) {
        HIPCHK(hipEventRecord(q->ev_src, q->s));
        HIPCHK(hipStreamWaitEvent(q->ds, q->ev_src, 0));
        q->ds_waits_src = true;
      }
      HIPCHK(hipMemcpyAsync(q->KA + off, r.src, r.n * G.kb, hipMemcpyDeviceToDevice, q->ds));
      const int rc = dispatch(q->KA + off, nullptr, nullptr, 1, r.n, r.n, r.dt, q->ds, false);
      if (rc != TSQS_OK) { q->broken = true; return rc; }
      hipEvent_t ev = nullptr;
      if (!q->ev_free.empty()) { ev = q->ev_free.back(); q->ev_free.pop_back(); }
      else HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      HIPCHK(hipEventRecord(ev, q->ds));
      q->direct.emplace_back(tk, ev);
      r.direct = true;
      r.state = 1;
      q->pending.pop_front();
      continue;
    }
    if (G.next_roots.size() >= kQRootsPerTick || q->free_ids.empty()) break;
    uint64_t off = 0;
    if (!arena_take(q, r.bytes, &off)) break;
    r.boff = off;
    r.id = q->free_ids.back();
    q->free_ids.pop_back();
    q->h_flag[r.id] = 0u;
    q->id_ticket[r.id] = tk;
    if (!G.waits_src) {
      // the source was written on the caller's stream before the submit
      HIPCHK(hipEventRecord(q->ev_src, q->s));
      HIPCHK(hipStreamWaitEvent(G.s, q->ev_src, 0));
      G.waits_src = true;
    }
    HIPCHK(hipMemcpyAsync(q->KA + off, r.src, r.n * G.kb, hipMemcpyDeviceToDevice, G.s));
    RootRec rr;
    rr.off = off / G.kb;
    rr.len = (uint32_t)r.n;
    rr.req = r.id;
    G.next_roots.push_back(rr);
    if (r.n > G.max_n) G.max_n = r.n;
    G.live++;
    r.state = 1;
    q->pending.pop_front();
  }
  return TSQS_OK;
}

int tick_dt(tsqs_queue *q, int dt) {
  QGroup &G = q->g[dt];
  switch (dt) {
    case TSQS_INT32: return queue_tick<0>(q, G);
    case TSQS_UINT32: return queue_tick<1>(q, G);
    case TSQS_INT64: return queue_tick<2>(q, G);
    case TSQS_UINT64: return queue_tick<3>(q, G);
    default: return queue_tick<4>(q, G);
  }
}

void queue_free(tsqs_queue *q) {
  for (int i = 0; i < 5; i++) group_free(q->g[i]);
  (void)hipFree(q->KA);
  (void)hipFree(q->SA);
  (void)hipFree(q->req_left);
  (void)hipFree(q->d_pos);
  (void)hipHostFree(q->h_flag);
  (void)hipHostFree(q->h_ring);
  if (q->ev_src) (void)hipEventDestroy(q->ev_src);
  for (auto &d : q->direct) (void)hipEventDestroy(d.second);
  for (hipEvent_t e : q->ev_free) (void)hipEventDestroy(e);
  q->direct.clear();
  q->ev_free.clear();
  if (q->ds) (void)hipStreamDestroy(q->ds);
}

}  // namespace

extern "C" {

int tsqs_queue_open(size_t budget_bytes, void *stream, tsqs_queue_t **out) {
  if (!out) return TSQS_EINVAL;
  *out = nullptr;
  if (budget_bytes < ((size_t)64 << 20)) return TSQS_EINVAL;
  tsqs_queue *q = new (std::nothrow) tsqs_queue();
  if (!q) return TSQS_ENOMEM;
  q->s = (hipStream_t)stream;
  int rc = TSQS_OK;
  auto fail = [&](int code) { queue_free(q); delete q; return code; };
  if (hipGetDevice(&q->dev) != hipSuccess) return fail(TSQS_EDEVICE);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, q->dev) != hipSuccess) return fail(TSQS_EDEVICE);
  q->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  q->lds_budget = prop.sharedMemPerBlock > 0 ? (size_t)prop.sharedMemPerBlock : 65536;
  // budget = two arenas + the tables of the three key widths a server mixes
  // (4-byte integer, 4-byte float, 8-byte integer), each sized for a full arena
  size_t arena = budget_bytes / 2;
  for (int it = 0; it < 4; it++) {
    const size_t t32 = group_table_bytes(arena / 4, queue_geom(TSQS_INT32, q->lds_budget).small_max,
                                         nullptr, nullptr, nullptr);
    const size_t t64 = group_table_bytes(arena / 8, queue_geom(TSQS_INT64, q->lds_budget).small_max,
                                         nullptr, nullptr, nullptr);
    const size_t tables = 2 * t32 + t64 + kQMaxReq * (sizeof(unsigned long long) + 4);
    if (tables >= budget_bytes / 2) return fail(TSQS_EINVAL);
    arena = ((budget_bytes - tables) / 2) / kArenaAlign * kArenaAlign;
  }
  q->arena_bytes = arena;
  size_t c0 = 0;
  if (grow(&q->KA, &c0, arena) != TSQS_OK) return fail(TSQS_ENOMEM);
  c0 = 0;
  if (grow(&q->SA, &c0, arena) != TSQS_OK) return fail(TSQS_ENOMEM);
  c0 = 0;
  if (grow(&q->req_left, &c0, (size_t)kQMaxReq) != TSQS_OK) return fail(TSQS_ENOMEM);
  if (hipHostMalloc(&q->h_flag, sizeof(unsigned int) * kQMaxReq,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return fail(TSQS_ENOMEM);
  std::memset(q->h_flag, 0, sizeof(unsigned int) * kQMaxReq);
  if (hipHostGetDevicePointer((void **)&q->d_flag, q->h_flag, 0) != hipSuccess) return fail(TSQS_EDEVICE);
  if (hipHostMalloc(&q->h_ring, sizeof(unsigned int) * kQMaxReq,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return fail(TSQS_ENOMEM);
  std::memset(q->h_ring, 0, sizeof(unsigned int) * kQMaxReq);
  if (hipHostGetDevicePointer((void **)&q->d_ring, q->h_ring, 0) != hipSuccess) return fail(TSQS_EDEVICE);
  c0 = 0;
  if (grow(&q->d_pos, &c0, (size_t)1) != TSQS_OK) return fail(TSQS_ENOMEM);
  if (hipMemset(q->d_pos, 0, sizeof(unsigned int)) != hipSuccess) return fail(TSQS_EDEVICE);
  if (hipEventCreateWithFlags(&q->ev_src, hipEventDisableTiming) != hipSuccess) return fail(TSQS_EDEVICE);
  if (hipStreamCreateWithFlags(&q->ds, hipStreamNonBlocking) != hipSuccess) return fail(TSQS_EDEVICE);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    q->direct_min = (uint64_t)g_opt.queue_direct;
  }
  q->id_ticket.assign(kQMaxReq, 0);
  q->free_ranges[0] = arena;
  q->free_ids.reserve(kQMaxReq);
  for (uint32_t i = 0; i < kQMaxReq; i++) q->free_ids.push_back(kQMaxReq - 1 - i);
  if ((rc = queue_fin_lds<0>(queue_geom(0, q->lds_budget))) != TSQS_OK) return fail(rc);
  if ((rc = queue_fin_lds<1>(queue_geom(1, q->lds_budget))) != TSQS_OK) return fail(rc);
  if ((rc = queue_fin_lds<2>(queue_geom(2, q->lds_budget))) != TSQS_OK) return fail(rc);
  if ((rc = queue_fin_lds<3>(queue_geom(3, q->lds_budget))) != TSQS_OK) return fail(rc);
  if ((rc = queue_fin_lds<4>(queue_geom(4, q->lds_budget))) != TSQS_OK) return fail(rc);
  *out = q;
  return TSQS_OK;
}

int tsqs_queue_submit(tsqs_queue_t *q, const void *d_src, size_t nmemb, int dt, uint64_t *ticket) {
  if (!q || !ticket) return TSQS_EINVAL;
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  if (!d_src || nmemb == 0 || nmemb > 0xFFFFFFFFull) return TSQS_EINVAL;
  if (((uintptr_t)d_src % dt_bytes(dt)) != 0) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  if (q->broken) return TSQS_EINTERNAL;
  QReq r;
  r.dt = dt;
  r.src = d_src;
  r.n = nmemb;
  r.bytes = (nmemb * dt_bytes(dt) + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
  if (r.bytes > q->arena_bytes) return TSQS_ENOMEM;
  const uint64_t tk = q->next_ticket++;
  if (nmemb == 1) {
    // one key is sorted: done without device work (its result is the source)
    r.state = 2;
    q->n_done++;
    q->reap.push_back(tk);
  }
  q->reqs.emplace(tk, r);
  if (nmemb > 1) q->pending.push_back(tk);
  *ticket = tk;
  return TSQS_OK;
}

int tsqs_queue_step(tsqs_queue_t *q) {
  if (!q) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  if (q->broken) return TSQS_EINTERNAL;
  if (hipSetDevice(q->dev) != hipSuccess) return TSQS_EDEVICE;
  collect_done(q);
  for (int dt = 0; dt < 5; dt++) q->g[dt].waits_src = false;
  q->ds_waits_src = false;
  int rc = admit(q);
  if (rc != TSQS_OK) return rc;
  for (int dt = 0; dt < 5; dt++) {
    QGroup &G = q->g[dt];
    if (!G.ready || (G.live == 0 && G.next_roots.empty())) continue;
    rc = tick_dt(q, dt);
    if (rc == TSQS_EAGAIN) continue;
    if (rc != TSQS_OK) return rc;
  }
  return TSQS_OK;
}

int tsqs_queue_poll(tsqs_queue_t *q, uint64_t ticket) {
  if (!q) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return TSQS_EINVAL;
  QReq &r = it->second;
  if (r.state == 1 && (r.direct || __atomic_load_n(&q->h_flag[r.id], __ATOMIC_ACQUIRE))) collect_done(q);
  return r.state;
}

int tsqs_queue_result(tsqs_queue_t *q, uint64_t ticket, void **d_keys, size_t *nmemb) {
  if (!q || !d_keys) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return TSQS_EINVAL;
  QReq &r = it->second;
  if (r.state == 1 && (r.direct || __atomic_load_n(&q->h_flag[r.id], __ATOMIC_ACQUIRE))) collect_done(q);
  if (r.state != 2) return TSQS_EAGAIN;
  *d_keys = r.n == 1 ? (void *)r.src : (void *)(q->KA + r.boff);
  if (nmemb) *nmemb = (size_t)r.n;
  return TSQS_OK;
}

int tsqs_queue_reap(tsqs_queue_t *q, uint64_t *tickets, size_t cap, size_t *count) {
  if (!q || !count || (cap && !tickets)) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  collect_done(q);
  size_t k = 0;
  while (k < cap && !q->reap.empty()) {
    tickets[k++] = q->reap.front();
    q->reap.pop_front();
  }
  *count = k;
  return TSQS_OK;
}

int tsqs_queue_release(tsqs_queue_t *q, uint64_t ticket) {
  if (!q) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return TSQS_EINVAL;
  QReq &r = it->second;
  if (r.state == 1 && (r.direct || __atomic_load_n(&q->h_flag[r.id], __ATOMIC_ACQUIRE))) collect_done(q);
  if (r.state != 2) return TSQS_EAGAIN;
  if (r.n > 1) {
    arena_give(q, r.boff, r.bytes);
    if (!r.direct) q->free_ids.push_back(r.id);
  }
  q->n_done--;
  q->reqs.erase(it);
  return TSQS_OK;
}

int tsqs_queue_cancel(tsqs_queue_t *q, uint64_t ticket) {
  if (!q) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return TSQS_EINVAL;
  QReq &r = it->second;
  if (r.state == 1) return TSQS_EAGAIN;        // its device work is enqueued
  if (r.state == 2) {
    // done: the same as a release (a one-key request may wait in the reap list)
    if (r.n > 1) {
      arena_give(q, r.boff, r.bytes);
      if (!r.direct) q->free_ids.push_back(r.id);
    }
    for (auto p = q->reap.begin(); p != q->reap.end(); ++p)
      if (*p == ticket) { q->reap.erase(p); break; }
    q->n_done--;
    q->reqs.erase(it);
    return TSQS_OK;
  }
  for (auto p = q->pending.begin(); p != q->pending.end(); ++p)
    if (*p == ticket) { q->pending.erase(p); break; }
  q->reqs.erase(it);
  return TSQS_OK;
}

int tsqs_queue_info(tsqs_queue_t *q, uint64_t *queued, uint64_t *running, uint64_t *done,
                    uint64_t *arena_used, uint64_t *arena_bytes) {
  if (!q) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  collect_done(q);
  uint64_t run = q->direct.size();
  for (int i = 0; i < 5; i++) run += q->g[i].live;
  if (queued) *queued = q->pending.size();
  if (running) *running = run;
  if (done) *done = q->n_done;
  if (arena_used) *arena_used = q->arena_used;
  if (arena_bytes) *arena_bytes = q->arena_bytes;
  return TSQS_OK;
}

int tsqs_queue_close(tsqs_queue_t *q) {
  if (!q) return TSQS_EINVAL;
  int rc = TSQS_OK;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    for (int i = 0; i < 5; i++)
      if (q->g[i].s && hipStreamSynchronize(q->g[i].s) != hipSuccess) rc = TSQS_EDEVICE;
    if (q->ds && hipStreamSynchronize(q->ds) != hipSuccess) rc = TSQS_EDEVICE;
    if (hipStreamSynchronize(q->s) != hipSuccess) rc = TSQS_EDEVICE;
    queue_free(q);
  }
  delete q;
  return rc;
}

}  // extern "C"

// ---- the entry point that allocates nothing ----------------------------------
//
// tsqs_sort_noalloc takes every device buffer of the call (the scratch copy of
// the keys and payloads, the level tables, the small-part and band slots, the
// statistics words) from one file-scope device array.  Its address is taken
// once per device with hipGetSymbolAddress, on the first call with that
// device current, and only that address is used afterwards: in host code the
// array's name is not a device address.  The level table is read back into
// static host arrays (the call holds the library mutex).

static __device__ __align__(256) unsigned char scratch[TSQS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
struct ScratchDev {
  bool ready = false;
  unsigned char *ptr = nullptr;     // device address of `scratch` on that device
  int cus = 256;
  size_t lds_budget = 65536;
};
ScratchDev g_scr[kMaxDevices];
LevelCtl g_scr_lvl[kMaxLevels];
unsigned long long g_scr_stats[kStripes * kStatWords + 16];

// The persistent schedule's ring and control words sit at the start of the
// array, at the same place for every call: a ring slot's sequence word must
// never have held anything but sequence words (cleared once at set-up).
constexpr size_t kScrQcap = 1u << 14;
constexpr size_t kScrRingBytes = kScrQcap * (sizeof(Task) + sizeof(unsigned long long)) +
                                 kQWords * sizeof(unsigned long long);

// Lays the buffers of a call out in [base, base + cap) (256-byte aligned
// pieces, after the ring); false if they do not fit.
bool carve(unsigned char *base, size_t cap, const WsNeed &nd, bool hasv, WsView *v) {
  v->seq = (unsigned long long *)base;
  v->ctl = v->seq + kScrQcap;
  v->task = (Task *)(v->ctl + kQWords);
  v->qcap = kScrQcap;
  size_t off = (kScrRingBytes + 255) & ~(size_t)255;
  auto take = [&](size_t bytes) -> unsigned char * {
    unsigned char *p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  v->S = take(nd.s_bytes);
  v->VS = hasv ? (uint32_t *)take(nd.v_elems * 4) : nullptr;
  v->VE = hasv ? (uint32_t *)take(nd.v_elems * 4) : nullptr;
  for (int i = 0; i < 2; i++) {
    v->seg[i] = (Seg *)take(nd.seg_cap * sizeof(Seg));
    v->ctr[i] = (unsigned long long *)take(nd.seg_cap * kCtrStride * sizeof(unsigned long long));
  }
  v->fin = (FinItem *)take(nd.slot_cap * sizeof(FinItem));
  v->finw = (FinItem *)take(nd.slot_cap * sizeof(FinItem));
  v->band = (FinItem *)take(nd.band_cap * sizeof(FinItem));
  v->big = (FinItem *)take(nd.big_cap * sizeof(FinItem));
  v->lvl = (LevelCtl *)take(sizeof(LevelCtl) * kMaxLevels);
  v->stats = (unsigned long long *)take(sizeof(unsigned long long) * (kStripes * kStatWords + 16));
  v->offs = nullptr;
  v->seg_cap = nd.seg_cap;
  v->slot_cap = nd.slot_cap;
  v->big_cap = nd.big_cap;
  v->parts = (TPart *)take(nd.part_cap * sizeof(TPart));
  v->pctr = (unsigned long long *)take(nd.part_cap * kCtrStride * sizeof(unsigned long long));
  v->hist = (uint32_t *)take(nd.hist_cap * 256 * sizeof(uint32_t));
  v->bands = (FinItem *)take(nd.lband_cap * sizeof(FinItem));
  v->sfin = (FinItem *)take(nd.sfin_cap * sizeof(FinItem));
  v->sfin_cap = nd.sfin_cap;
  v->part_cap = nd.part_cap;
  v->hist_cap = nd.hist_cap;
  v->band_cap = nd.lband_cap;
  return off <= cap && nd.qcap <= kScrQcap;
}

}  // namespace

extern "C" int tsqs_sort_noalloc(void *d_keys, uint32_t *d_vals, size_t nmemb, int dt, void *stream) {
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  if (nmemb <= 1) return TSQS_OK;
  if (!d_keys) return TSQS_EINVAL;
  if (nmemb > TSQS_NOALLOC_MAX_KEYS) return TSQS_ESCRATCH;
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return TSQS_EDEVICE;
  ScratchDev &sd = g_scr[dev];
  if (!sd.ready) {
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    sd.ptr = (unsigned char *)ptr;
    sd.cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    sd.lds_budget = prop.sharedMemPerBlock > 0 ? (size_t)prop.sharedMemPerBlock : 65536;
    // the ring's sequence and control words start at zero (a kernel, on the
    // caller's stream, before any use)
    hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, (hipStream_t)stream, (unsigned long long *)sd.ptr,
                       (uint64_t)(kScrQcap + kQWords));
    HIPCHK(hipGetLastError());
    sd.ready = true;
  }
  g_last.valid = false;
  const bool hv = d_vals != nullptr;
  const FinGeom geo = geom_any(dt, sd.lds_budget, hv);
  const WsNeed nd = ws_need((uint64_t)nmemb, 1, dt_bytes(dt), hv, geo.small_max, false);
  CallEnv env;
  if (!carve(sd.ptr, TSQS_NOALLOC_SCRATCH_BYTES, nd, hv, &env.v)) return TSQS_ESCRATCH;
  env.cus = sd.cus;
  env.lds_budget = sd.lds_budget;
  env.h_lvl = g_scr_lvl;
  env.h_stats = g_scr_stats;
  env.ev = nullptr;
  CallArgs a;
  a.keys = d_keys; a.vals = d_vals; a.h_offs = nullptr; a.nroots = 1; a.n = nmemb;
  a.max_root = nmemb; a.s = (hipStream_t)stream;
  return sort_any(dt, env, a);
}

extern "C" {

int tsqs_sort(void *d_keys, size_t nmemb, int dt, void *stream) {
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  if (nmemb <= 1) return TSQS_OK;
  if (!d_keys) return TSQS_EINVAL;
  if (nmemb > 0xFFFFFFFFull) return TSQS_EINVAL;
  return dispatch(d_keys, nullptr, nullptr, 1, (uint64_t)nmemb, (uint64_t)nmemb, dt,
                  (hipStream_t)stream);
}

int tsqs_sort_pairs(void *d_keys, uint32_t *d_vals, size_t nmemb, int dt, void *stream) {
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  if (nmemb <= 1) return TSQS_OK;
  if (!d_keys || !d_vals) return TSQS_EINVAL;
  if (nmemb > 0xFFFFFFFFull) return TSQS_EINVAL;
  return dispatch(d_keys, d_vals, nullptr, 1, (uint64_t)nmemb, (uint64_t)nmemb, dt,
                  (hipStream_t)stream);
}

int tsqs_sort_records(void *d_keys, void *d_records, size_t rec_bytes, void *d_out, size_t nmemb,
                      int dt, void *stream) {
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  if (nmemb == 0) return TSQS_OK;
  if (!d_keys || !d_records || rec_bytes == 0 || rec_bytes > kMaxRecBytes) return TSQS_EINVAL;
  if (nmemb > 0xFFFFFFFFull) return TSQS_EINVAL;
  const size_t total = nmemb * rec_bytes;
  if (d_out == d_records) d_out = nullptr;
  if (d_out) {
    const uintptr_t a = (uintptr_t)d_records, b = (uintptr_t)d_out;
    if (a < b + total && b < a + total) return TSQS_EINVAL;   // overlapping, not identical
  }
  hipStream_t s = (hipStream_t)stream;
  if (nmemb == 1) {
    if (d_out) HIPCHK(hipMemcpyAsync(d_out, d_records, rec_bytes, hipMemcpyDeviceToDevice, s));
    return TSQS_OK;
  }
  std::lock_guard<std::mutex> lk(g_rec_mu);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0) return TSQS_EDEVICE;
  if ((size_t)dev >= g_rec.size()) g_rec.resize((size_t)dev + 1);
  RecWs &r = g_rec[(size_t)dev];
  int rc;
  if (r.idx_cap < nmemb || (!d_out && r.tmp_cap < total)) {
    // the index and the staging buffer are regrown only after the last call
    std::lock_guard<std::mutex> lk2(g_mu);
    if ((size_t)dev < g_ws.size() && g_ws[(size_t)dev].init && (rc = ws_quiesce(g_ws[(size_t)dev])) != TSQS_OK)
      return rc;
  }
  if ((rc = grow(&r.idx, &r.idx_cap, nmemb)) != TSQS_OK) return rc;
  if ((rc = grow(&r.err, &r.err_cap, 1)) != TSQS_OK) return rc;
  int cus = 256;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      cus = prop.multiProcessorCount;
  }
  const uint64_t blocks_needed = (nmemb + kRecNT - 1) / kRecNT;
  const int grid = (int)(blocks_needed < (uint64_t)(8 * cus) ? blocks_needed : (uint64_t)(8 * cus));
  hipLaunchKernelGGL(k_rec_iota, dim3(grid), dim3(kRecNT), 0, s, r.idx, (uint64_t)nmemb, r.err);
  HIPCHK(hipGetLastError());
  // the keys with the index as payload: the paper's sorted pointer array
  if ((rc = dispatch(d_keys, r.idx, nullptr, 1, (uint64_t)nmemb, (uint64_t)nmemb, dt, s)) != TSQS_OK)
    return rc;
  void *dst = d_out;
  if (!dst) {
    if ((rc = grow(&r.tmp, &r.tmp_cap, total)) != TSQS_OK) return rc;
    dst = r.tmp;
  }
  unsigned int *err = nullptr;
  {
    std::lock_guard<std::mutex> lk2(g_mu);
    err = (unsigned int *)(g_ws[(size_t)dev].stats + kStripes * kStatWords);
  }
  const uintptr_t al = (uintptr_t)d_records | (uintptr_t)dst | (uintptr_t)rec_bytes;
  const size_t wsz = (al & 15u) == 0 ? 16 : (al & 7u) == 0 ? 8 : (al & 3u) == 0 ? 4 : 1;
  const uint64_t gtiles = (total / wsz + (uint64_t)kRecNT * kRecU - 1) / ((uint64_t)kRecNT * kRecU);
  const int ggrid = (int)(gtiles < (uint64_t)(16 * cus) ? gtiles : (uint64_t)(16 * cus));
  if ((al & 15u) == 0)
    hipLaunchKernelGGL(k_rec_gather<uint4>, dim3(ggrid), dim3(kRecNT), 0, s, (const uint4 *)d_records,
                       (uint4 *)dst, r.idx, (uint64_t)nmemb, (uint32_t)(rec_bytes / 16), err);
  else if ((al & 7u) == 0)
    hipLaunchKernelGGL(k_rec_gather<uint2>, dim3(ggrid), dim3(kRecNT), 0, s, (const uint2 *)d_records,
                       (uint2 *)dst, r.idx, (uint64_t)nmemb, (uint32_t)(rec_bytes / 8), err);
  else if ((al & 3u) == 0)
    hipLaunchKernelGGL(k_rec_gather<uint32_t>, dim3(ggrid), dim3(kRecNT), 0, s, (const uint32_t *)d_records,
                       (uint32_t *)dst, r.idx, (uint64_t)nmemb, (uint32_t)(rec_bytes / 4), err);
  else
    hipLaunchKernelGGL(k_rec_gather<uint8_t>, dim3(ggrid), dim3(kRecNT), 0, s, (const uint8_t *)d_records,
                       (uint8_t *)dst, r.idx, (uint64_t)nmemb, (uint32_t)rec_bytes, err);
  HIPCHK(hipGetLastError());
  if (!d_out) HIPCHK(hipMemcpyAsync(d_records, r.tmp, total, hipMemcpyDeviceToDevice, s));
  {
    // the call ends after the gather: later calls wait for it, and its
    // statistics (and an index that was not a permutation) are read after it
    std::lock_guard<std::mutex> lk2(g_mu);
    Workspace &w = g_ws[(size_t)dev];
    HIPCHK(hipEventRecord(w.done, s));
    w.done_rec = true;
    w.last_stream = s;
  }
  return TSQS_OK;
}

int tsqs_sort_batch(void *d_keys, uint32_t *d_vals, const uint64_t *h_offsets, size_t nseg,
                    int dt, void *stream) {
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  if (nseg == 0) return TSQS_OK;
  if (!h_offsets) return TSQS_EINVAL;
  if (nseg >= (1ull << 24)) return TSQS_EINVAL;
  if (h_offsets[0] != 0) return TSQS_EINVAL;
  uint64_t max_root = 0;
  for (size_t j = 0; j < nseg; j++) {
    if (h_offsets[j + 1] < h_offsets[j]) return TSQS_EINVAL;
    uint64_t len = h_offsets[j + 1] - h_offsets[j];
    if (len > 0xFFFFFFFFull) return TSQS_EINVAL;
    if (len > max_root) max_root = len;
  }
  const uint64_t total = h_offsets[nseg];
  if (max_root <= 1) return TSQS_OK;
  if (!d_keys) return TSQS_EINVAL;
  return dispatch(d_keys, d_vals, h_offsets, nseg, total, max_root, dt, (hipStream_t)stream);
}

int tsqs_graph_create(void *d_keys, uint32_t *d_vals, size_t nmemb, const uint64_t *h_offsets,
                      size_t nseg, int dt, tsqs_graph_t **out) {
  if (!out) return TSQS_EINVAL;
  *out = nullptr;
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  if (!d_keys) return TSQS_EINVAL;
  uint64_t n = nmemb, max_root = nmemb;
  size_t nroots = 1;
  if (h_offsets) {
    if (nseg == 0 || nseg >= (1ull << 24) || h_offsets[0] != 0) return TSQS_EINVAL;
    max_root = 0;
    for (size_t j = 0; j < nseg; j++) {
      if (h_offsets[j + 1] < h_offsets[j]) return TSQS_EINVAL;
      const uint64_t len = h_offsets[j + 1] - h_offsets[j];
      if (len > 0xFFFFFFFFull) return TSQS_EINVAL;
      if (len > max_root) max_root = len;
    }
    if (h_offsets[nseg] != nmemb) return TSQS_EINVAL;
    nroots = nseg;
  } else if (nmemb > 0xFFFFFFFFull) {
    return TSQS_EINVAL;
  }
  if (n < 2 || max_root < 2) return TSQS_EINVAL;   // nothing to sort: no graph
  const size_t kb = dt_bytes(dt);
  if (((uintptr_t)d_keys % kb) != 0 || ((uintptr_t)d_vals % 4) != 0) return TSQS_EINVAL;
  tsqs_graph *g = new (std::nothrow) tsqs_graph();
  if (!g) return TSQS_ENOMEM;
  auto fail = [&](int code) {
    if (g->cs) (void)hipStreamSynchronize(g->cs);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->done) (void)hipEventDestroy(g->done);
    free_ws(g->w);
    if (g->cs) (void)hipStreamDestroy(g->cs);
    delete g;
    (void)hipGetLastError();
    return code;
  };
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipGetDevice(&g->dev) != hipSuccess) return fail(TSQS_EDEVICE);
  if (hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking) != hipSuccess) return fail(TSQS_EDEVICE);
  if (hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess) return fail(TSQS_EDEVICE);
  // buffers and their first clears, then the offsets, before the capture starts
  int rc = ensure_static(g->w, g->dev, g->cs);
  if (rc != TSQS_OK) return fail(rc);
  const bool hv = d_vals != nullptr;
  const FinGeom geo = geom_any(dt, g->w.lds_budget, hv);
  WsNeed nd = ws_need(n, nroots, kb, hv, geo.small_max, h_offsets != nullptr);
  if (g_opt.debug) nd.dbg = 3 * (size_t)n;
  CallEnv env;
  if ((rc = ws_grow(g->w, nd, hv, &env.v, g->cs)) != TSQS_OK) return fail(rc);
  if (h_offsets &&
      hipMemcpy(env.v.offs, h_offsets, (nroots + 1) * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess)
    return fail(TSQS_EDEVICE);
  if (hipStreamSynchronize(g->cs) != hipSuccess) return fail(TSQS_EDEVICE);
  env.cus = g->w.cus;
  env.lds_budget = g->w.lds_budget;
  env.h_lvl = g->w.h_lvl;
  env.h_stats = g->w.h_stats;
  env.ev = nullptr;      // no per-level timing events in a graph
  env.done = nullptr;    // the launch records the graph's own event
  CallArgs a;
  a.keys = d_keys; a.vals = d_vals; a.h_offs = h_offsets; a.nroots = nroots; a.n = n;
  a.max_root = max_root; a.s = g->cs; a.offs_ready = true;
  const LastCall saved = g_last;
  if (hipStreamBeginCapture(g->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(TSQS_EDEVICE);
  rc = sort_any(dt, env, a);
  g->lc = g_last;
  g_last = saved;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(g->cs, &graph);
  g->graph = graph;
  if (rc != TSQS_OK) return fail(rc);
  if (e != hipSuccess || !graph) return fail(TSQS_EDEVICE);
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) return fail(TSQS_EDEVICE);
  g->lc.done = g->done;
  g->lc.ev = nullptr;
  *out = g;
  return TSQS_OK;
}

int tsqs_graph_launch(tsqs_graph_t *g, void *stream) {
  if (!g) return TSQS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // launches of one graph share its buffers: a launch on another stream starts
  // after the previous one
  if (g->launched && g->last != s) HIPCHK(hipStreamWaitEvent(s, g->done, 0));
  HIPCHK(hipGraphLaunch(g->exec, s));
  HIPCHK(hipEventRecord(g->done, s));
  g->last = s;
  g->launched = true;
  return TSQS_OK;
}

int tsqs_graph_stats(tsqs_graph_t *g, tsqs_stats_t *out) {
  if (!g || !out) return TSQS_EINVAL;
  if (!g->launched) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  const LastCall saved = g_last;
  g_last = g->lc;
  g_last.s = g->last;
  const int rc = stats_of_last(out);
  g_last = saved;
  return rc;
}

int tsqs_graph_destroy(tsqs_graph_t *g) {
  if (!g) return TSQS_EINVAL;
  int rc = TSQS_OK;
  if (g->launched && hipEventSynchronize(g->done) != hipSuccess) rc = TSQS_EDEVICE;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->done) (void)hipEventDestroy(g->done);
  free_ws(g->w);
  if (g->cs) (void)hipStreamDestroy(g->cs);
  delete g;
  return rc;
}

void tsqs_free_storage(void) {
  std::lock_guard<std::mutex> lr(g_rec_mu);   // same order as tsqs_sort_records
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) cur = -1;
  for (size_t i = 0; i < g_ws.size(); i++) {
    if (!g_ws[i].init) continue;
    if (hipSetDevice((int)i) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    free_ws(g_ws[i]);
  }
  for (size_t i = 0; i < g_rec.size(); i++) {
    RecWs &r = g_rec[i];
    if (!r.idx && !r.tmp && !r.err) continue;
    if (hipSetDevice((int)i) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    (void)hipFree(r.idx); (void)hipFree(r.tmp); (void)hipFree(r.err);
    r = RecWs();
  }
  if (cur >= 0) (void)hipSetDevice(cur);
  g_ws.clear();
  g_rec.clear();
}

int tsqs_set_option(int key, int64_t v) {
  std::lock_guard<std::mutex> lk(g_mu);
  switch (key) {
    case TSQS_OPT_SMALL_MAX: if (v < 16 || v > 8192) return TSQS_EINVAL; g_opt.small_max = v; return TSQS_OK;
    case TSQS_OPT_SAMPLES: if (v < 3 || v > 63 || !(v & 1)) return TSQS_EINVAL; g_opt.samples = v; return TSQS_OK;
    case TSQS_OPT_DEPTH_FACTOR: if (v < 1 || v > 4) return TSQS_EINVAL; g_opt.depth_factor = v; return TSQS_OK;
    case TSQS_OPT_PIVOT_MODE: if (v < 0 || v > 1) return TSQS_EINVAL; g_opt.pivot_mode = v; return TSQS_OK;
    case TSQS_OPT_SEED: g_opt.seed = v; return TSQS_OK;
    case TSQS_OPT_TIMING: g_opt.timing = v ? 1 : 0; return TSQS_OK;
    case TSQS_OPT_PART_GRID: if (v < 0 || v > 65536) return TSQS_EINVAL; g_opt.part_grid = v; return TSQS_OK;
    case TSQS_OPT_FINISH_GRID: if (v < 0 || v > 65536) return TSQS_EINVAL; g_opt.finish_grid = v; return TSQS_OK;
    case TSQS_OPT_FINISH_ALGO: if (v < 0 || v > 3) return TSQS_EINVAL; g_opt.finish_algo = v; return TSQS_OK;
    case TSQS_OPT_PRESORT: g_opt.presort = v ? 1 : 0; return TSQS_OK;
    case TSQS_OPT_SCHEDULE: if (v < 0 || v > 1) return TSQS_EINVAL; g_opt.schedule = v; return TSQS_OK;
    case TSQS_OPT_ITER_CAP: if (v < 0) return TSQS_EINVAL; g_opt.iter_cap = v; return TSQS_OK;
    case TSQS_OPT_QUEUE_DIRECT: if (v < 0 || v > 0xFFFFFFFFll) return TSQS_EINVAL; g_opt.queue_direct = v; return TSQS_OK;
    case TSQS_OPT_PART_THREADS1: if (v != kPartNT1 && v != 2 * kPartNT1) return TSQS_EINVAL; g_opt.part_threads1 = v; return TSQS_OK;
    case TSQS_OPT_PART_THREADS2: if (v != kPartNT2 && v != 2 * kPartNT2) return TSQS_EINVAL; g_opt.part_threads2 = v; return TSQS_OK;
    case TSQS_OPT_WORKSPACE_CAP: if (v < 0) return TSQS_EINVAL; g_opt.workspace_cap = v; return TSQS_OK;
    case TSQS_OPT_DEBUG: if (v < 0 || v > 3) return TSQS_EINVAL; g_opt.debug = v; return TSQS_OK;
    default: return TSQS_EUNSUPPORTED;
  }
}

int64_t tsqs_get_option(int key) {
  std::lock_guard<std::mutex> lk(g_mu);
  switch (key) {
    case TSQS_OPT_SMALL_MAX: return g_opt.small_max;
    case TSQS_OPT_SAMPLES: return g_opt.samples;
    case TSQS_OPT_DEPTH_FACTOR: return g_opt.depth_factor;
    case TSQS_OPT_PIVOT_MODE: return g_opt.pivot_mode;
    case TSQS_OPT_SEED: return g_opt.seed;
    case TSQS_OPT_TIMING: return g_opt.timing;
    case TSQS_OPT_PART_GRID: return g_opt.part_grid;
    case TSQS_OPT_FINISH_GRID: return g_opt.finish_grid;
    case TSQS_OPT_FINISH_ALGO: return g_opt.finish_algo;
    case TSQS_OPT_PRESORT: return g_opt.presort;
    case TSQS_OPT_SCHEDULE: return g_opt.schedule;
    case TSQS_OPT_ITER_CAP: return g_opt.iter_cap;
    case TSQS_OPT_QUEUE_DIRECT: return g_opt.queue_direct;
    case TSQS_OPT_PART_THREADS1: return g_opt.part_threads1;
    case TSQS_OPT_PART_THREADS2: return g_opt.part_threads2;
    case TSQS_OPT_WORKSPACE_CAP: return g_opt.workspace_cap;
    case TSQS_OPT_DEBUG: return g_opt.debug;
    default: return INT64_MIN;
  }
}

int tsqs_get_stats(tsqs_stats_t *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!out) return TSQS_EINVAL;
  return stats_of_last(out);
}

const char *tsqs_strerror(int code) {
  switch (code) {
    case TSQS_OK: return "success";
    case TSQS_EINVAL: return "invalid argument";
    case TSQS_ENOMEM: return "device workspace allocation failed";
    case TSQS_EDEVICE: return "HIP runtime error";
    case TSQS_EUNSUPPORTED: return "unsupported dtype or option";
    case TSQS_EINTERNAL: return "internal capacity or level limit exceeded";
    case TSQS_EAGAIN: return "not yet (request not done, or no room yet)";
    case TSQS_ESCRATCH: return "request exceeds the fixed scratch of tsqs_sort_noalloc";
    default: return "unknown error code";
  }
}

int tsqs_version(void) { return 3; }

}  // extern "C"


extern "C" {

int tsqs_autotune(int dt, int with_payload, size_t n, const uint64_t *h_offsets, size_t nseg,
                  void *stream, tsqs_tune_t *out) {
  if (!dtype_ok(dt)) return TSQS_EUNSUPPORTED;
  if (n < 2 || n > ((size_t)1 << 36)) return TSQS_EINVAL;
  if (h_offsets) {
    if (nseg == 0 || nseg >= (1ull << 24) || h_offsets[0] != 0 || h_offsets[nseg] != n) return TSQS_EINVAL;
    for (size_t j = 0; j < nseg; j++)
      if (h_offsets[j + 1] < h_offsets[j] || h_offsets[j + 1] - h_offsets[j] > 0xFFFFFFFFull) return TSQS_EINVAL;
  } else if (n > 0xFFFFFFFFull) {
    return TSQS_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t kb = (dt == TSQS_INT64 || dt == TSQS_UINT64) ? 8 : 4;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TSQS_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return TSQS_EDEVICE;
  const int64_t cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  Options saved;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    saved = g_opt;
  }
  // tuning cache: the same architecture and shape tuned before
  const char *cache = std::getenv("TSQS_TUNE_CACHE");
  if (cache && !*cache) cache = nullptr;
  std::string ckey;
  if (cache) {
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    char kb_[160];
    std::snprintf(kb_, sizeof kb_, "%s dt=%d v=%d b=%d lg=%u", arch.c_str(), dt, with_payload ? 1 : 0,
                  h_offsets ? 1 : 0, ceil_log2(n));
    ckey = kb_;
    Options o = saved;
    double md = 0.0, mb = 0.0;
    bool hit;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      hit = tune_cache_find(cache, ckey, &o, &md, &mb);
    }
    if (hit) {
      {
        std::lock_guard<std::mutex> lk(g_mu);
        g_opt = o;
      }
      if (out) {
        std::memset(out, 0, sizeof *out);
        out->small_max = o.small_max; out->samples = o.samples; out->part_grid = o.part_grid;
        out->finish_grid = o.finish_grid; out->finish_algo = o.finish_algo;
        out->part_threads1 = o.part_threads1; out->part_threads2 = o.part_threads2;
        out->ms_default = md; out->ms_best = mb; out->trials = 0;
      }
      return TSQS_OK;
    }
  }
  unsigned char *keys0 = nullptr, *keys = nullptr;
  uint32_t *vals = nullptr;
  int rc = TSQS_OK;
  if (hipMalloc(&keys0, n * kb) != hipSuccess || hipMalloc(&keys, n * kb) != hipSuccess ||
      (with_payload && hipMalloc(&vals, n * sizeof(uint32_t)) != hipSuccess)) {
    (void)hipGetLastError();
    rc = TSQS_ENOMEM;
  }
  if (rc == TSQS_OK) {
    hipLaunchKernelGGL(k_tune_keys, dim3(4 * (unsigned)cus), dim3(256), 0, s, (void *)keys0, (uint64_t)n,
                       (int)kb, (uint64_t)0x7E57ull);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = TSQS_EDEVICE;
  }
  // fastest of two timed sorts after one untimed, with options o
  auto trial = [&](const Options &o, double *ms) -> int {
    {
      std::lock_guard<std::mutex> lk(g_mu);
      g_opt = o;
    }
    double best = 1e30;
    for (int rep = 0; rep < 3; rep++) {
      HIPCHK(hipMemcpyAsync(keys, keys0, n * kb, hipMemcpyDeviceToDevice, s));
      if (with_payload) hipLaunchKernelGGL(k_tune_iota, dim3(4 * (unsigned)cus), dim3(256), 0, s, vals, (uint64_t)n);
      HIPCHK(hipStreamSynchronize(s));
      const auto t0 = std::chrono::steady_clock::now();
      int r;
      if (h_offsets) r = tsqs_sort_batch(keys, with_payload ? vals : nullptr, h_offsets, nseg, dt, s);
      else if (with_payload) r = tsqs_sort_pairs(keys, vals, n, dt, s);
      else r = tsqs_sort(keys, n, dt, s);
      if (r != TSQS_OK) return r;
      HIPCHK(hipStreamSynchronize(s));
      const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (rep > 0 && t < best) best = t;
    }
    *ms = best;
    return TSQS_OK;
  };
  Options best = saved;
  double ms_default = 0.0, ms_best = 0.0;
  uint32_t trials = 0;
  if (rc == TSQS_OK) rc = trial(best, &ms_default);
  ms_best = ms_default;
  trials = 1;
  // one parameter at a time, keeping the best so far
  auto try_value = [&](int64_t Options::*field, int64_t v) {
    if (rc != TSQS_OK || best.*field == v) return;
    Options o = best;
    o.*field = v;
    double ms = 0.0;
    rc = trial(o, &ms);
    trials++;
    if (rc == TSQS_OK && ms < ms_best) { ms_best = ms; best = o; }
  };
  for (int64_t t : {2048, 4096, 8192}) try_value(&Options::small_max, t);
  for (int64_t v : {31, 63}) try_value(&Options::samples, v);
  for (int64_t m : {2, 4, 5, 6, 8}) try_value(&Options::part_grid, m * cus);
  for (int64_t m : {8, 16, 32}) try_value(&Options::finish_grid, m * cus);
  for (int64_t a : {0, 1, 2, 3}) try_value(&Options::finish_algo, a);
  // workgroup size against keys per thread (the same chunk of keys)
  for (int64_t t : {(int64_t)kPartNT1, (int64_t)2 * kPartNT1}) try_value(&Options::part_threads1, t);
  for (int64_t t : {(int64_t)kPartNT2, (int64_t)2 * kPartNT2}) try_value(&Options::part_threads2, t);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_opt = rc == TSQS_OK ? best : saved;
  }
  (void)hipFree(keys0);
  (void)hipFree(keys);
  (void)hipFree(vals);
  if (rc == TSQS_OK && out) {
    out->small_max = best.small_max;
    out->samples = best.samples;
    out->part_grid = best.part_grid;
    out->finish_grid = best.finish_grid;
    out->finish_algo = best.finish_algo;
    out->part_threads1 = best.part_threads1;
    out->part_threads2 = best.part_threads2;
    out->ms_default = ms_default;
    out->ms_best = ms_best;
    out->trials = trials;
    out->reserved = 0;
  }
  if (rc == TSQS_OK && cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_append(cache, ckey, best, ms_default, ms_best);
  }
  return rc;
}

}  // extern "C"


