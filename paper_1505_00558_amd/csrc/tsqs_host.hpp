// tsqs_host.hpp -- host-side state shared by the translation units of libtsqs.
//
// The library is built from tsqs_host.hip (C ABI, options, workspace, records,
// autotuner, serving queue) and one tsqs_dt.hip object per key type (the
// launch schedule and its kernel instances for that type), compiled in
// parallel.  This header holds what both sides need: options, the workspace
// and its per-call view, the small-part geometry, and the per-key-type entry
// points.
#pragma once

#include "tsqs.h"
#include "tsqs_queue.h"
#include "tsqs_kernels.hpp"
#include "tsqs_persist.hpp"

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace tsqs {
namespace host {

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return TSQS_EDEVICE;         \
  } while (0)

// Workgroups of the small-part finish per compute unit (default grid): many
// more than fit at once, so that parts of unequal size balance over the CUs.
constexpr int kFinGridPerCu = 32;

struct Options {
  int64_t small_max = 8192;
  int64_t samples = 63;
  int64_t depth_factor = 2;
  int64_t pivot_mode = 0;
  int64_t seed = 0x5EED1505;
  int64_t timing = 0;
  int64_t part_grid = 0;
  int64_t finish_grid = 0;
  int64_t finish_algo = 3;
  int64_t presort = 1;
  int64_t schedule = 0;        // TSQS_OPT_SCHEDULE
  int64_t iter_cap = 0;        // TSQS_OPT_ITER_CAP (0: the default)
  int64_t queue_direct = 1 << 22;   // TSQS_OPT_QUEUE_DIRECT
  int64_t part_threads1 = kPartNT1;  // TSQS_OPT_PART_THREADS1
  int64_t part_threads2 = kPartNT2;  // TSQS_OPT_PART_THREADS2
  int64_t workspace_cap = 0;         // TSQS_OPT_WORKSPACE_CAP (bytes, 0: none)
  int64_t debug = 0;                 // TSQS_OPT_DEBUG
};

constexpr unsigned long long kDefaultIterCap = 1ull << 23;

// Device buffers of one call: the scratch copy of the keys (and payloads), the
// level tables and the small-part / band slots.  Capacities in elements.
struct WsView {
  void *S = nullptr;
  uint32_t *VS = nullptr, *VE = nullptr;
  Seg *seg[2] = {nullptr, nullptr};
  unsigned long long *ctr[2] = {nullptr, nullptr};
  FinItem *fin = nullptr, *finw = nullptr, *band = nullptr, *big = nullptr;
  LevelCtl *lvl = nullptr;
  unsigned long long *stats = nullptr;   // kStripes x kStatWords, then 16 words of flags
  uint64_t *offs = nullptr;
  size_t seg_cap = 0, slot_cap = 0, big_cap = 0;
  // persistent schedule: task ring, its control words, the part pool
  Task *task = nullptr;
  unsigned long long *seq = nullptr, *ctl = nullptr;
  TPart *parts = nullptr;
  unsigned long long *pctr = nullptr;
  uint32_t *hist = nullptr;
  FinItem *bands = nullptr;
  FinItem *sfin = nullptr;
  size_t qcap = 0, part_cap = 0, hist_cap = 0, band_cap = 0, sfin_cap = 0;
  unsigned int *dbg = nullptr;          // debug shadows (3 n words), or null
};

// Element counts a call needs (see ws_need).
struct WsNeed {
  size_t s_bytes = 0, v_elems = 0, seg_cap = 0, slot_cap = 0, band_cap = 0, big_cap = 0, offs = 0;
  size_t qcap = 0, part_cap = 0, hist_cap = 0, lband_cap = 0, sfin_cap = 0;   // persistent schedule
  size_t dbg = 0;                      // debug shadow words (TSQS_OPT_DEBUG): 3 n, else 0
};

// Per-device workspace of the allocating entry points: grows to the largest
// request seen and is kept between calls (the paper's persistent buffer).
struct Workspace {
  bool init = false;
  int cus = 0;
  size_t lds_budget = 0;
  size_t s_bytes = 0;
  void *S = nullptr;
  size_t v_cap = 0;
  uint32_t *VS = nullptr, *VE = nullptr;
  size_t seg_cap = 0;
  Seg *seg[2] = {nullptr, nullptr};
  unsigned long long *ctr[2] = {nullptr, nullptr};
  size_t slot_cap = 0, band_cap = 0, big_cap = 0;
  FinItem *fin = nullptr, *finw = nullptr, *band = nullptr, *big = nullptr;
  LevelCtl *lvl = nullptr;
  unsigned long long *stats = nullptr;
  size_t off_cap = 0;
  uint64_t *offs = nullptr;
  LevelCtl *h_lvl = nullptr;             // pinned
  unsigned long long *h_stats = nullptr; // pinned
  hipEvent_t ev[2 * kMaxLevels];
  bool ev_ok = false;
  // persistent schedule
  size_t qcap = 0, part_cap = 0, hist_cap = 0, lband_cap = 0, sfin_cap = 0;
  FinItem *sfin = nullptr;
  Task *task = nullptr;
  unsigned long long *seq = nullptr, *ctl = nullptr;
  TPart *parts = nullptr;
  unsigned long long *pctr = nullptr;
  uint32_t *hist = nullptr;
  FinItem *bands = nullptr;
  size_t dbg_cap = 0;
  unsigned int *dbg = nullptr;
  // the last call's completion: later calls on another stream wait for it,
  // buffers are freed or regrown only after it
  hipEvent_t done = nullptr;
  bool done_rec = false;
  hipStream_t last_stream = nullptr;
};

// What the statistics of the last call need (read when they are asked for).
struct LastCall {
  bool valid = false;
  hipEvent_t done = nullptr;             // or null: synchronise the stream
  hipStream_t s = nullptr;
  const LevelCtl *d_lvl = nullptr;
  const unsigned long long *d_stats = nullptr;
  LevelCtl *h_lvl = nullptr;
  unsigned long long *h_stats = nullptr;
  hipEvent_t *ev = nullptr;              // per-level timing events, or null
  uint32_t levels = 0;
  bool roots_small = false;
  uint64_t n = 0;
  uint32_t kb = 4, vb = 0;
  uint32_t schedule = 0;
};

// Where a call's device buffers come from and where its level table is read back.
struct CallEnv {
  WsView v;
  int cus = 256;
  size_t lds_budget = 65536;
  LevelCtl *h_lvl = nullptr;             // host copy of the level table (kMaxLevels)
  unsigned long long *h_stats = nullptr; // host copy of the statistics words
  hipEvent_t *ev = nullptr;              // 2 * kMaxLevels timing events, or null
  hipEvent_t done = nullptr;             // recorded at the end of the call, or null
};

struct CallArgs {
  void *keys = nullptr;
  uint32_t *vals = nullptr;
  const uint64_t *h_offs = nullptr;  // batch offsets (host), or null for one array
  size_t nroots = 1;
  uint64_t n = 0;
  uint64_t max_root = 0;
  hipStream_t s = nullptr;
  bool offs_ready = false;           // the batch offsets are already in the workspace
};

extern Options g_opt;
extern std::mutex g_mu;
extern uint64_t g_calls;
extern LastCall g_last;

template <typename T>
int grow(T **p, size_t *cap, size_t need, size_t elem = sizeof(T)) {
  if (*cap >= need) return TSQS_OK;
  if (*p) { (void)hipFree(*p); *p = nullptr; *cap = 0; }
  void *q = nullptr;
  if (hipMalloc(&q, need * elem) != hipSuccess) { (void)hipGetLastError(); return TSQS_ENOMEM; }
  *p = static_cast<T *>(q);
  *cap = need;
  return TSQS_OK;
}

inline size_t lds_pad_host(size_t x) { return x + (x >> 5); }

inline uint32_t ceil_log2(uint64_t x) {
  uint32_t l = 0;
  while (l < 64 && (1ull << l) < x) l++;
  return l;
}

inline uint32_t mix32(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return (uint32_t)(z ^ (z >> 31));
}

inline bool dtype_ok(int dt) { return dt >= TSQS_INT32 && dt <= TSQS_FLOAT32; }
inline size_t dt_bytes(int dt) { return (dt == TSQS_INT64 || dt == TSQS_UINT64) ? 8 : 4; }

// Small-part geometry of a key type: one wave sorts up to wave_max keys, the
// workgroup up to small_max (the option, clipped to what registers and LDS
// hold); fin_lds is the dynamic LDS of the finish kernel.
struct FinGeom {
  uint32_t small_max, wave_max;
  size_t fin_lds;
};

template <int DT, bool HASV>
FinGeom fin_geom(size_t lds_budget, int64_t small_opt) {
  using B = typename Codec<DT>::B;
  using RT = typename Rec<B, HASV>::T;
  const uint32_t me = (uint32_t)max_e<RT>();
  uint32_t wave_max = 64 * me;
  while (wave_max > 64 && kFinNW * lds_pad_host(wave_max) * sizeof(RT) > lds_budget) wave_max >>= 1;
  uint32_t wg_max = kFinNT * me;
  while (wg_max > wave_max && lds_pad_host(wg_max) * sizeof(RT) > lds_budget) wg_max >>= 1;
  uint32_t small_max = (uint32_t)small_opt;
  if (small_max > wg_max) small_max = wg_max;
  if (small_max < 16) small_max = 16;
  uint32_t P = 1;
  while (P < small_max) P <<= 1;
  size_t fin_lds = lds_pad_host(P) * sizeof(RT);
  if (kFinNW * lds_pad_host(wave_max) * sizeof(RT) > fin_lds) fin_lds = kFinNW * lds_pad_host(wave_max) * sizeof(RT);
  return FinGeom{small_max, wave_max, fin_lds};
}

// Buffer sizes of a call of n keys in nroots arrays with small parts of up to
// small_max keys.
inline size_t pow2_at_least(size_t x) {
  size_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

inline WsNeed ws_need(uint64_t n, size_t nroots, size_t kb, bool hasv, uint32_t small_max, bool batch) {
  WsNeed w;
  w.s_bytes = (size_t)n * kb;
  w.v_elems = hasv ? (size_t)n : 0;
  w.seg_cap = (size_t)(n / (small_max + 1)) + 2;
  w.slot_cap = 4 * w.seg_cap + nroots;   // 4 child slots per part, then the roots
  w.band_cap = 3 * w.seg_cap;
  w.big_cap = 2 * (size_t)(n / kBandChunk) + 16;
  w.offs = batch ? nroots + 1 : 0;
  // persistent schedule: every part of the recursion below the parts it is
  // given (at most about 2 n / small_max), the roots, and the ring with room
  // for every task that can be waiting at once
  w.part_cap = 3 * (size_t)(n / (small_max + 1)) + nroots + 1024;
  w.hist_cap = w.part_cap < 4096 ? w.part_cap : 4096;
  w.lband_cap = (size_t)(n / kBandChunk) + 64;
  w.sfin_cap = 4 * w.part_cap;   // at most four small children per planned part
  const size_t tasks = 2 * (size_t)(n / (4096ull * kTaskChunks)) + 2 * (size_t)(n / (kSelChunk * kTaskChunks)) +
                       (size_t)(n / kBandChunk) + w.part_cap + 4096;
  w.qcap = pow2_at_least(2 * tasks);
  return w;
}

// Per-key-type entry points (tsqs_dt.hip, one object per type).
template <int DT> int sort_dt(const CallEnv &env, const CallArgs &a, bool hasv);
template <int DT> FinGeom geom_dt(size_t lds_budget, bool hasv);

}  // namespace host
}  // namespace tsqs
