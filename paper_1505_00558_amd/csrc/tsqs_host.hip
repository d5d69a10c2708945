// tsqs_host.hip -- host driver and C ABI of libtsqs (see include/tsqs.h).
//
// One call = one schedule on the caller's stream:
//   k_reset, [upload of batch offsets], k_init (roots: pivot or small item),
//   then per level d: k_partition(d), k_plan(d), k_finish(d),
// launched without host synchronisation for the number of levels a median
// split needs (ceil(log2(n / small_max)) + 2); the stream is then synchronised
// once, and only if parts remain (bad pivots, the depth-limit path) more levels
// are launched, eight at a time.
#include "tsqs.h"
#include "tsqs_kernels.hpp"
#include "tsqs_records.hpp"
#include "tsqs_queue.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <climits>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

using namespace tsqs;

namespace {

// Arrays of at least this many keys synchronise once after the presortedness
// check (about 10-20 us) so that an array found in order skips the level schedule.
constexpr uint64_t kPresortSyncMin = 1ull << 24;

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
};

struct Workspace {
  bool init = false;
  int cus = 0;
  size_t s_bytes = 0;
  void *S = nullptr;
  size_t v_cap = 0;
  uint32_t *VS = nullptr, *VE = nullptr;
  size_t lds_budget = 0;
  size_t seg_cap = 0;
  Seg *seg[2] = {nullptr, nullptr};
  unsigned long long *ctr[2] = {nullptr, nullptr};
  size_t slot_cap = 0, band_cap = 0, big_cap = 0;
  FinItem *fin = nullptr, *finw = nullptr, *band = nullptr, *big = nullptr;
  LevelCtl *lvl = nullptr;
  unsigned long long *stats = nullptr;   // kStripes x kStatWords, then one word of error flags
  size_t off_cap = 0;
  uint64_t *offs = nullptr;
  LevelCtl *h_lvl = nullptr;             // pinned
  unsigned long long *h_stats = nullptr; // pinned
  hipEvent_t ev[2 * kMaxLevels];
  bool ev_ok = false;
};

std::mutex g_mu;

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
Options g_opt;
std::vector<Workspace> g_ws;
tsqs_stats_t g_stats;
bool g_have_stats = false;
uint64_t g_calls = 0;

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return TSQS_EDEVICE;         \
  } while (0)

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

void free_ws(Workspace &w) {
  (void)hipFree(w.S); (void)hipFree(w.VS); (void)hipFree(w.VE);
  for (int i = 0; i < 2; i++) { (void)hipFree(w.seg[i]); (void)hipFree(w.ctr[i]); }
  (void)hipFree(w.fin); (void)hipFree(w.finw); (void)hipFree(w.band); (void)hipFree(w.big);
  (void)hipFree(w.lvl); (void)hipFree(w.stats); (void)hipFree(w.offs);
  (void)hipHostFree(w.h_lvl); (void)hipHostFree(w.h_stats);
  if (w.ev_ok) for (int i = 0; i < 2 * kMaxLevels; i++) (void)hipEventDestroy(w.ev[i]);
  w = Workspace();
}

int ensure_static(Workspace &w, int dev) {
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
  w.init = true;
  return TSQS_OK;
}

size_t lds_pad_host(size_t x) { return x + (x >> 5); }

uint32_t ceil_log2(uint64_t x) {
  uint32_t l = 0;
  while (l < 64 && (1ull << l) < x) l++;
  return l;
}

uint32_t mix32(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return (uint32_t)(z ^ (z >> 31));
}

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

template <int DT, bool HASV>
int run_t(Workspace &w, void *keys, uint32_t *vals, const uint64_t *h_offs, size_t nroots,
          uint64_t n, uint64_t max_root, hipStream_t s) {
  using B = typename Codec<DT>::B;
  const size_t kb = sizeof(B);
  if (((uintptr_t)keys % kb) != 0 || ((uintptr_t)vals % 4) != 0) return TSQS_EINVAL;
  const FinGeom geo = fin_geom<DT, HASV>(w.lds_budget, g_opt.small_max);
  const uint32_t small_max = geo.small_max, wave_max = geo.wave_max;

  // workspace sizes
  const size_t seg_cap = (size_t)(n / (small_max + 1)) + 2;
  const size_t slot_cap = 4 * seg_cap + nroots;   // 4 child slots per part, then the roots
  const size_t big_cap = 2 * (size_t)(n / kBandChunk) + 16;
  int rc;
  {
    size_t cap_bytes = w.s_bytes;
    void *S = w.S;
    if ((rc = grow<unsigned char>((unsigned char **)&S, &cap_bytes, (size_t)n * kb)) != TSQS_OK) return rc;
    w.S = S; w.s_bytes = cap_bytes;
  }
  if (HASV) {
    size_t c1 = w.v_cap, c2 = w.v_cap;
    if ((rc = grow(&w.VS, &c1, (size_t)n)) != TSQS_OK) return rc;
    if ((rc = grow(&w.VE, &c2, (size_t)n)) != TSQS_OK) return rc;
    w.v_cap = c1 < c2 ? c1 : c2;
  }
  if (w.seg_cap < seg_cap) {
    for (int i = 0; i < 2; i++) {
      size_t a = w.seg_cap, b = w.seg_cap * kCtrStride;
      if ((rc = grow(&w.seg[i], &a, seg_cap)) != TSQS_OK) return rc;
      if ((rc = grow(&w.ctr[i], &b, seg_cap * kCtrStride)) != TSQS_OK) return rc;
    }
    w.seg_cap = seg_cap;
  }
  if (w.slot_cap < slot_cap) {
    size_t a = w.slot_cap, b = w.slot_cap;
    if ((rc = grow(&w.fin, &a, slot_cap)) != TSQS_OK) return rc;
    if ((rc = grow(&w.finw, &b, slot_cap)) != TSQS_OK) return rc;
    w.slot_cap = slot_cap;
  }
  if ((rc = grow(&w.band, &w.band_cap, 3 * seg_cap)) != TSQS_OK) return rc;
  if ((rc = grow(&w.big, &w.big_cap, big_cap)) != TSQS_OK) return rc;
  if (h_offs) {
    if ((rc = grow(&w.offs, &w.off_cap, nroots + 1)) != TSQS_OK) return rc;
    HIPCHK(hipMemcpyAsync(w.offs, h_offs, (nroots + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  }
  if (g_opt.timing && !w.ev_ok) {
    for (int i = 0; i < 2 * kMaxLevels; i++) HIPCHK(hipEventCreate(&w.ev[i]));
    w.ev_ok = true;
  }

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

  const int part_grid = g_opt.part_grid > 0 ? (int)g_opt.part_grid : 4 * w.cus;
  const int fin_grid = g_opt.finish_grid > 0 ? (int)g_opt.finish_grid : 8 * w.cus;
  const int plan_grid = 4 * w.cus;
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
  int init_grid = (int)(waves_init < (size_t)(4 * w.cus) ? waves_init : (size_t)(4 * w.cus));
  if (init_grid < 1) init_grid = 1;

  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, c);
  if (c.pre) {
    const uint64_t pre_chunks = (n + (uint64_t)kPreNT * kPreRows - 1) / ((uint64_t)kPreNT * kPreRows);
    const int scan_grid = (int)(pre_chunks < (uint64_t)(8 * w.cus) ? pre_chunks : (uint64_t)(8 * w.cus));
    hipLaunchKernelGGL((k_presort_scan<DT>), dim3(scan_grid), dim3(kPreNT), 0, s, c);
    hipLaunchKernelGGL((k_presort_reverse<DT, HASV>), dim3(8 * w.cus), dim3(kPreNT), 0, s, c);
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
    unsigned int *hp = (unsigned int *)(w.h_stats + kStripes * kStatWords + 8);
    HIPCHK(hipMemcpyAsync(hp, c.pre, 2 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hp[0] != 0u && hp[1] == 0u) target = 0;
  }
  if (target > kMaxLevels - 1) target = kMaxLevels - 1;
  for (;;) {
    for (; d < target; d++) {
      const bool idle = d == 0 && roots_small;
      if (g_opt.timing) HIPCHK(hipEventRecord(w.ev[2 * d], s));
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
      if (g_opt.timing) HIPCHK(hipEventRecord(w.ev[2 * d + 1], s));
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
    HIPCHK(hipMemcpyAsync(w.h_lvl, w.lvl, sizeof(LevelCtl) * (size_t)(d + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(w.h_stats, w.stats, sizeof(unsigned long long) * (kStripes * kStatWords + 1),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*(unsigned int *)(w.h_stats + kStripes * kStatWords)) return TSQS_EINTERNAL;
    if ((w.h_lvl[d].packed >> 40) == 0) break;
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
    const unsigned long long *sp = w.h_stats + (size_t)i * kStatWords;
    st.fallback_parts += sp[kStFallback];
    st.small_parts += sp[kStSmallParts];
    st.small_keys += sp[kStSmallKeys];
    st.band_keys += sp[kStBandKeys];
    st.presorted += (uint32_t)(sp[kStPresorted] + sp[kStPresortedRoots]);
  }
  for (int i = 0; i < d; i++)
    if (w.h_lvl[i].packed >> 40) st.max_depth = (uint32_t)i;
  for (int i = 0; i < d && i < TSQS_MAX_LEVELS; i++) {
    st.level_keys[i] = w.h_lvl[i].keys;
    st.level_parts[i] = (uint32_t)(w.h_lvl[i].packed >> 40);
    st.partition_bytes += 2ull * w.h_lvl[i].keys * (kb + (HASV ? 4 : 0));
    if (!(i == 0 && roots_small)) st.partition_launches++;
    if (g_opt.timing) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, w.ev[2 * i], w.ev[2 * i + 1]));
      st.level_ms[i] = ms;
      st.partition_ms += ms;
    }
  }
  g_have_stats = true;
  return TSQS_OK;
}

int dispatch(void *keys, uint32_t *vals, const uint64_t *h_offs, size_t nroots, uint64_t n,
             uint64_t max_root, int dt, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0) return TSQS_EDEVICE;
  if ((size_t)dev >= g_ws.size()) g_ws.resize((size_t)dev + 1);
  Workspace &w = g_ws[(size_t)dev];
  int rc = ensure_static(w, dev);
  if (rc != TSQS_OK) return rc;
  g_have_stats = false;
  const bool hv = vals != nullptr;
  switch (dt) {
    case TSQS_INT32: return hv ? run_t<0, true>(w, keys, vals, h_offs, nroots, n, max_root, s)
                               : run_t<0, false>(w, keys, vals, h_offs, nroots, n, max_root, s);
    case TSQS_UINT32: return hv ? run_t<1, true>(w, keys, vals, h_offs, nroots, n, max_root, s)
                                : run_t<1, false>(w, keys, vals, h_offs, nroots, n, max_root, s);
    case TSQS_INT64: return hv ? run_t<2, true>(w, keys, vals, h_offs, nroots, n, max_root, s)
                               : run_t<2, false>(w, keys, vals, h_offs, nroots, n, max_root, s);
    case TSQS_UINT64: return hv ? run_t<3, true>(w, keys, vals, h_offs, nroots, n, max_root, s)
                                : run_t<3, false>(w, keys, vals, h_offs, nroots, n, max_root, s);
    case TSQS_FLOAT32: return hv ? run_t<4, true>(w, keys, vals, h_offs, nroots, n, max_root, s)
                                 : run_t<4, false>(w, keys, vals, h_offs, nroots, n, max_root, s);
    default: return TSQS_EUNSUPPORTED;
  }
}

bool dtype_ok(int dt) { return dt >= TSQS_INT32 && dt <= TSQS_FLOAT32; }

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
    HIPCHK(hipStreamSynchronize(s));
    return TSQS_OK;
  }
  std::lock_guard<std::mutex> lk(g_rec_mu);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0) return TSQS_EDEVICE;
  if ((size_t)dev >= g_rec.size()) g_rec.resize((size_t)dev + 1);
  RecWs &r = g_rec[(size_t)dev];
  int rc;
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
  const uintptr_t al = (uintptr_t)d_records | (uintptr_t)dst | (uintptr_t)rec_bytes;
  const size_t wsz = (al & 15u) == 0 ? 16 : (al & 7u) == 0 ? 8 : (al & 3u) == 0 ? 4 : 1;
  const uint64_t gtiles = (total / wsz + (uint64_t)kRecNT * kRecU - 1) / ((uint64_t)kRecNT * kRecU);
  const int ggrid = (int)(gtiles < (uint64_t)(16 * cus) ? gtiles : (uint64_t)(16 * cus));
  if ((al & 15u) == 0)
    hipLaunchKernelGGL(k_rec_gather<uint4>, dim3(ggrid), dim3(kRecNT), 0, s, (const uint4 *)d_records,
                       (uint4 *)dst, r.idx, (uint64_t)nmemb, (uint32_t)(rec_bytes / 16), r.err);
  else if ((al & 7u) == 0)
    hipLaunchKernelGGL(k_rec_gather<uint2>, dim3(ggrid), dim3(kRecNT), 0, s, (const uint2 *)d_records,
                       (uint2 *)dst, r.idx, (uint64_t)nmemb, (uint32_t)(rec_bytes / 8), r.err);
  else if ((al & 3u) == 0)
    hipLaunchKernelGGL(k_rec_gather<uint32_t>, dim3(ggrid), dim3(kRecNT), 0, s, (const uint32_t *)d_records,
                       (uint32_t *)dst, r.idx, (uint64_t)nmemb, (uint32_t)(rec_bytes / 4), r.err);
  else
    hipLaunchKernelGGL(k_rec_gather<uint8_t>, dim3(ggrid), dim3(kRecNT), 0, s, (const uint8_t *)d_records,
                       (uint8_t *)dst, r.idx, (uint64_t)nmemb, (uint32_t)rec_bytes, r.err);
  HIPCHK(hipGetLastError());
  if (!d_out) HIPCHK(hipMemcpyAsync(d_records, r.tmp, total, hipMemcpyDeviceToDevice, s));
  unsigned int h_err = 0;
  HIPCHK(hipMemcpyAsync(&h_err, r.err, sizeof h_err, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return h_err ? TSQS_EINTERNAL : TSQS_OK;
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
    default: return INT64_MIN;
  }
}

int tsqs_get_stats(tsqs_stats_t *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!out) return TSQS_EINVAL;
  if (!g_have_stats) return TSQS_EINVAL;
  *out = g_stats;
  return TSQS_OK;
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
    default: return "unknown error code";
  }
}

int tsqs_version(void) { return 1; }

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
  for (int64_t m : {2, 4, 8}) try_value(&Options::part_grid, m * cus);
  for (int64_t m : {2, 4, 8}) try_value(&Options::finish_grid, m * cus);
  for (int64_t a : {0, 1, 2, 3}) try_value(&Options::finish_algo, a);
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
    out->ms_default = ms_default;
    out->ms_best = ms_best;
    out->trials = trials;
    out->reserved = 0;
  }
  return rc;
}

}  // extern "C"

#include "tsqs_queue_impl.hpp"
