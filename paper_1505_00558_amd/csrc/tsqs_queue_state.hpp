// tsqs_queue_state.hpp -- state of the serving queue of include/tsqs_queue.h.
//
// Layout.  Two arenas of equal size, A_K (keys) and A_S (the scratch copy a
// part uses at odd depths), carved first-fit in 256-byte units: a request of n
// keys of b bytes holds [o, o + n*b) in both.  Per key type ("group") there is
// one set of level tables, sized for an arena full of that type, and a tick
// counter; tick t uses level index t mod kMaxLevels (the tables' parity and the
// kernels' buffer choice only need t's parity, and kMaxLevels is even).
//
// Requests of at least TSQS_OPT_QUEUE_DIRECT keys (read when the queue opens)
// skip the ticks: the single-array schedule sorts each in place in the arena on
// the queue's direct stream, one after another, and an event per request marks
// it done.  They hold arena space but no device request id.
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

#pragma once

#include "tsqs_host.hpp"

namespace tsqs {
namespace host {

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
  uint32_t id = 0;         // device request id (requests sorted by the ticks)
  int state = 0;           // 0 queued, 1 running, 2 done
  bool direct = false;     // sorted by the single-array schedule on the direct stream
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

}  // namespace host
}  // namespace tsqs

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
  std::unordered_map<uint64_t, tsqs::host::QReq> reqs;
  uint64_t next_ticket = 1;
  uint64_t n_done = 0;
  std::deque<uint64_t> reap;                  // done, not yet reported by tsqs_queue_reap
  tsqs::host::QGroup g[5];
  // requests of at least direct_min keys (0: none) are sorted by the
  // single-array schedule on stream ds; in flight: (ticket, completion event)
  uint64_t direct_min = 0;
  hipStream_t ds = nullptr;
  bool ds_waits_src = false;
  std::deque<std::pair<uint64_t, hipEvent_t>> direct;
  std::vector<hipEvent_t> ev_free;
  bool broken = false;
};


namespace tsqs {
namespace host {
// One tick of a key type's group (tsqs_dt.hip).
template <int DT> int queue_tick(tsqs_queue *q, QGroup &G);
template <int DT> int queue_fin_lds(const FinGeom &geo);
}  // namespace host
}  // namespace tsqs
