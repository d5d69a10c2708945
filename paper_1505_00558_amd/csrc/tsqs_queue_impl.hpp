// tsqs_queue_impl.hpp -- the serving queue of include/tsqs_queue.h (part of the
// tsqs_host.hip translation unit: it shares its helpers and kernel instances).
//
// Layout.  Two arenas of equal size, A_K (keys) and A_S (the scratch copy a
// part uses at odd depths), carved first-fit in 256-byte units: a request of n
// keys of b bytes holds [o, o + n*b) in both.  Per key type ("group") there is
// one set of level tables, sized for an arena full of that type, and a tick
// counter; tick t uses level index t mod kMaxLevels (the tables' parity and the
// kernels' buffer choice only need t's parity, and kMaxLevels is even).
//
// A tick of a group: clear the counters of the next level index, add the roots
// admitted since the last tick (k_init, which also sets each request's count of
// keys not yet final), then k_partition / k_plan / k_finish on every part of
// every live request of that type.  Finished small parts and filled bands
// subtract their keys from the request's count; the kernel thread that reaches
// zero raises the request's flag in host-mapped memory and appends the request
// to a host-mapped completion ring, which the host reads from its cursor on (so
// finding completions costs nothing per running request).  Each group runs on
// a stream of its own (default priority), so ticks of different key types
// overlap on the device; at most kInFlight ticks of a group are enqueued and
// not yet finished.

namespace {

constexpr uint32_t kQMaxReq = 1u << 16;       // live requests (device request ids)
constexpr uint32_t kQRootsPerTick = 2048;     // roots one tick admits per group
constexpr int kInFlight = 3;                  // enqueued, unfinished ticks per group
constexpr size_t kArenaAlign = 256;

struct QReq {
  int dt = 0;
  const void *src = nullptr;
  uint64_t n = 0;
  uint64_t boff = 0;       // byte offset in both arenas
  uint64_t bytes = 0;      // reserved bytes (rounded)
  uint32_t id = 0;         // device request id
  int state = 0;           // 0 queued, 1 running, 2 done
};

struct QGroup {
  bool ready = false;
  int dt = 0;
  size_t kb = 0;
  FinGeom geo{};
  size_t seg_cap = 0, slot_cap = 0, big_cap = 0;
  Seg *seg[2] = {nullptr, nullptr};
  unsigned long long *ctr[2] = {nullptr, nullptr};
  FinItem *fin = nullptr, *finw = nullptr, *band = nullptr, *big = nullptr;
  LevelCtl *lvl = nullptr;
  unsigned long long *stats = nullptr;   // kStripes x kStatWords, then the error word
  RootRec *d_roots[kInFlight] = {nullptr, nullptr, nullptr};
  RootRec *h_roots[kInFlight] = {nullptr, nullptr, nullptr};   // pinned staging
  unsigned int *h_err = nullptr;                               // pinned, kInFlight words
  hipEvent_t ev[kInFlight];
  bool ev_used[kInFlight] = {false, false, false};
  bool ev_made = false;
  hipStream_t s = nullptr;          // the group's own stream
  bool waits_src = false;           // the stream already waits for this step's sources
  uint64_t tick = 0;
  uint64_t max_n = 0;
  uint64_t live = 0;                // admitted and not yet seen done
  std::vector<RootRec> next_roots;
};

}  // namespace

struct tsqs_queue {
  std::mutex mu;
  int dev = 0;
  hipStream_t s = nullptr;
  int cus = 256;
  size_t lds_budget = 65536;
  size_t arena_bytes = 0, arena_used = 0;
  unsigned char *KA = nullptr, *SA = nullptr;
  std::map<uint64_t, uint64_t> free_ranges;   // offset -> length, in bytes
  unsigned long long *req_left = nullptr;     // device, kQMaxReq
  unsigned int *h_flag = nullptr;             // host-mapped, kQMaxReq
  unsigned int *d_flag = nullptr;             // device alias of h_flag
  unsigned int *h_ring = nullptr;             // host-mapped completion ring, kQMaxReq
  unsigned int *d_ring = nullptr;             // device alias of h_ring
  unsigned int *d_pos = nullptr;              // device: completions so far
  uint64_t ring_cur = 0;                      // host read cursor
  std::vector<uint64_t> id_ticket;            // device request id -> ticket
  hipEvent_t ev_src = nullptr;                // sources ready on the caller's stream
  std::vector<uint32_t> free_ids;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, QReq> reqs;
  uint64_t next_ticket = 1;
  uint64_t n_done = 0;
  std::deque<uint64_t> reap;                  // done, not yet reported by tsqs_queue_reap
  QGroup g[5];
  bool broken = false;
};

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

template <int DT>
FinGeom geom_of(size_t lds) { return fin_geom<DT, false>(lds, g_opt.small_max); }

FinGeom geom_dt(int dt, size_t lds) {
  switch (dt) {
    case TSQS_INT32: return geom_of<0>(lds);
    case TSQS_UINT32: return geom_of<1>(lds);
    case TSQS_INT64: return geom_of<2>(lds);
    case TSQS_UINT64: return geom_of<3>(lds);
    default: return geom_of<4>(lds);
  }
}

size_t dt_bytes(int dt) { return (dt == TSQS_INT64 || dt == TSQS_UINT64) ? 8 : 4; }

int group_init(tsqs_queue *q, int dt) {
  QGroup &G = q->g[dt];
  if (G.ready) return TSQS_OK;
  G.dt = dt;
  G.kb = dt_bytes(dt);
  G.geo = geom_dt(dt, q->lds_budget);
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

template <int DT>
int launch_tick(tsqs_queue *q, QGroup &G) {
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

int tick_dt(tsqs_queue *q, int dt) {
  QGroup &G = q->g[dt];
  switch (dt) {
    case TSQS_INT32: return launch_tick<0>(q, G);
    case TSQS_UINT32: return launch_tick<1>(q, G);
    case TSQS_INT64: return launch_tick<2>(q, G);
    case TSQS_UINT64: return launch_tick<3>(q, G);
    default: return launch_tick<4>(q, G);
  }
}

template <int DT>
int set_fin_lds(const FinGeom &geo) {
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

void queue_free(tsqs_queue *q) {
  for (int i = 0; i < 5; i++) group_free(q->g[i]);
  (void)hipFree(q->KA);
  (void)hipFree(q->SA);
  (void)hipFree(q->req_left);
  (void)hipFree(q->d_pos);
  (void)hipHostFree(q->h_flag);
  (void)hipHostFree(q->h_ring);
  if (q->ev_src) (void)hipEventDestroy(q->ev_src);
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
    const size_t t32 = group_table_bytes(arena / 4, geom_dt(TSQS_INT32, q->lds_budget).small_max,
                                         nullptr, nullptr, nullptr);
    const size_t t64 = group_table_bytes(arena / 8, geom_dt(TSQS_INT64, q->lds_budget).small_max,
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
  q->id_ticket.assign(kQMaxReq, 0);
  q->free_ranges[0] = arena;
  q->free_ids.reserve(kQMaxReq);
  for (uint32_t i = 0; i < kQMaxReq; i++) q->free_ids.push_back(kQMaxReq - 1 - i);
  if ((rc = set_fin_lds<0>(geom_dt(0, q->lds_budget))) != TSQS_OK) return fail(rc);
  if ((rc = set_fin_lds<1>(geom_dt(1, q->lds_budget))) != TSQS_OK) return fail(rc);
  if ((rc = set_fin_lds<2>(geom_dt(2, q->lds_budget))) != TSQS_OK) return fail(rc);
  if ((rc = set_fin_lds<3>(geom_dt(3, q->lds_budget))) != TSQS_OK) return fail(rc);
  if ((rc = set_fin_lds<4>(geom_dt(4, q->lds_budget))) != TSQS_OK) return fail(rc);
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
  if (r.state == 1 && __atomic_load_n(&q->h_flag[r.id], __ATOMIC_ACQUIRE)) collect_done(q);
  return r.state;
}

int tsqs_queue_result(tsqs_queue_t *q, uint64_t ticket, void **d_keys, size_t *nmemb) {
  if (!q || !d_keys) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return TSQS_EINVAL;
  QReq &r = it->second;
  if (r.state == 1 && __atomic_load_n(&q->h_flag[r.id], __ATOMIC_ACQUIRE)) collect_done(q);
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
  if (r.state == 1 && __atomic_load_n(&q->h_flag[r.id], __ATOMIC_ACQUIRE)) collect_done(q);
  if (r.state != 2) return TSQS_EAGAIN;
  if (r.n > 1) {
    arena_give(q, r.boff, r.bytes);
    q->free_ids.push_back(r.id);
  }
  q->n_done--;
  q->reqs.erase(it);
  return TSQS_OK;
}

int tsqs_queue_info(tsqs_queue_t *q, uint64_t *queued, uint64_t *running, uint64_t *done,
                    uint64_t *arena_used, uint64_t *arena_bytes) {
  if (!q) return TSQS_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  collect_done(q);
  uint64_t run = 0;
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
    if (hipStreamSynchronize(q->s) != hipSuccess) rc = TSQS_EDEVICE;
    queue_free(q);
  }
  delete q;
  return rc;
}

}  // extern "C"
