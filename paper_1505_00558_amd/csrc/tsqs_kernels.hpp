// tsqs_kernels.hpp -- gfx950 kernels of the three-way partition sort.
//
// The method is the recursion of Triple State QuickSort (Muqaddas, arXiv
// 1505.00558, SIII): pick a pivot from samples, split a part into keys < p,
// keys == p and keys > p, put the == p keys in a middle band that is final and
// never compared again, recurse on the two sides.  The paper's single-threaded
// hole-juggling scan (SIII.A-F) is not used; on the GPU the recursion runs as
// data-parallel passes over every active part, one or two recursion levels per
// read and write of the keys:
//
//   k_partition  every chunk of every part at this level.  A chunk is a
//                window of 32 keys per thread (16 / 8 for wider elements) from
//                the 128-byte line of the part's first key, read with 16-byte
//                loads by a 512-thread workgroup for one-level passes (loaded
//                straight into LDS while the previous chunk is processed) and a
//                256-thread one for two-level passes; integer keys compared as
//                themselves, float32 keys as order-preserving codes; ranks from
//                64-lane ballots + mbcnt; per-wave scalar cursors and one
//                reservation per chunk.
//                One-level parts are split by their pivot with a left and a
//                right cursor, and the keys of each side are counted against
//                that side's pivot; two-level parts (whose class sizes that
//                counting gave) get their < and > regions placed exactly and
//                each region split by its own pivot with two cursors, so one
//                pass does two levels (with payloads, the payloads of the
//                three bands' keys are staged for the band fills).  The keys
//                move to the other buffer (ping-pong K <-> S).
//   k_plan       one wave per part just partitioned: reads the final counters,
//                writes the equal bands and the small children into fixed
//                slots (no list atomics), and for large children picks the
//                pivots of the next two levels from one sorted sample of up to
//                63 keys (the exact median by radix select once the depth limit
//                is reached); the workgroup then reserves all its next-level
//                parts with one atomic.
//   k_finish     small parts are sorted in registers and LDS: a per-thread
//                sorting network, bitonic merging across the lanes of a wave
//                (lane exchanges, no LDS), then merge-path merging in LDS (or
//                alternatives: a bitonic network throughout, merge-path merging
//                from the per-thread runs on): one wave per part up to 2048
//                keys, the 256-thread workgroup above; bands write the pivot
//                value (equality means identical bits) and the staged payloads.
//
// Buffers: each part records whether its keys are in K or in S.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace tsqs {

constexpr int kWave = 64;
// partition workgroups: one-level passes 512 threads, two-level passes 256
// (measured: the two-level pass, with more synchronisation per key, gains from
// smaller workgroups, four per CU; the one-level pass from larger ones)
constexpr int kPartNT1 = 512, kPartNT2 = 256;
constexpr int kPlanNT = 256;
constexpr int kPlanNW = kPlanNT / kWave;
constexpr int kFinNT = 256;
constexpr int kFinNW = kFinNT / kWave;
constexpr int kPNT = 256;                  // threads of a persistent-schedule workgroup
constexpr int kPNW = kPNT / kWave;
constexpr uint32_t kTaskChunks = 4;        // chunks per partition / select task
constexpr uint32_t kSelChunk = 8192;       // keys per select chunk
constexpr uint32_t kSelInline = 1u << 16;  // exact pivots of parts up to this size: one wave
constexpr uint32_t kBandChunk = 1u << 16;
constexpr int kMaxLevels = 192;
constexpr unsigned long long kTileMask = (1ull << 40) - 1;
constexpr int kCtrStride = 64;   // u64 words between part counters: four 128-byte lines each
constexpr int kStripes = 64;     // statistics counters are spread over this many lines
constexpr int kStatWords = 16;
enum { kStFallback = 0, kStSmallParts = 1, kStSmallKeys = 2, kStBandKeys = 3, kStPresorted = 4,
       kStPresortedRoots = 5 };
constexpr uint32_t kErrSegCap = 1, kErrFinCap = 2, kErrLevel = 4, kErrCount = 8;
constexpr uint32_t kErrQueue = 16;   // persistent schedule: task ring or part pool full
constexpr uint32_t kErrIter = 32;    // persistent schedule: a workgroup reached its iteration cap
constexpr uint32_t kErrShadow = 128; // debug shadows: a slot written twice by one part's pass,
                                     // a store over a final slot, a slot finalised twice or never

// ---- order-preserving codes (compares are done on these, never on floats) --

template <int DT> struct Codec;
// C / ckey / cpiv: what the partition pass compares.  Integers compare as
// themselves (signed compares for signed keys, against the pivot decoded from
// its code: the same order as the codes, without encoding every key); float32
// keys compare as codes.
template <> struct Codec<0> {  // int32: flip the sign bit
  using B = uint32_t;
  using C = int32_t;
  __device__ static inline B enc(B x) { return x ^ 0x80000000u; }
  __device__ static inline B dec(B u) { return u ^ 0x80000000u; }
  __device__ static inline C ckey(B x) { return (int32_t)x; }
  __device__ static inline C cpiv(uint64_t code) { return (int32_t)((uint32_t)code ^ 0x80000000u); }
};
template <> struct Codec<1> {  // uint32
  using B = uint32_t;
  using C = uint32_t;
  __device__ static inline B enc(B x) { return x; }
  __device__ static inline B dec(B u) { return u; }
  __device__ static inline C ckey(B x) { return x; }
  __device__ static inline C cpiv(uint64_t code) { return (uint32_t)code; }
};
template <> struct Codec<2> {  // int64
  using B = uint64_t;
  using C = int64_t;
  __device__ static inline B enc(B x) { return x ^ 0x8000000000000000ull; }
  __device__ static inline B dec(B u) { return u ^ 0x8000000000000000ull; }
  __device__ static inline C ckey(B x) { return (int64_t)x; }
  __device__ static inline C cpiv(uint64_t code) { return (int64_t)(code ^ 0x8000000000000000ull); }
};
template <> struct Codec<3> {  // uint64
  using B = uint64_t;
  using C = uint64_t;
  __device__ static inline B enc(B x) { return x; }
  __device__ static inline B dec(B u) { return u; }
  __device__ static inline C ckey(B x) { return x; }
  __device__ static inline C cpiv(uint64_t code) { return code; }
};
template <> struct Codec<4> {  // float32 bits, IEEE totalOrder: negatives reversed
  using B = uint32_t;
  using C = uint32_t;
  __device__ static inline B enc(B x) {
    return x ^ ((uint32_t)((int32_t)x >> 31) | 0x80000000u);
  }
  __device__ static inline B dec(B u) {
    return u ^ (~(uint32_t)((int32_t)u >> 31) | 0x80000000u);
  }
  __device__ static inline C ckey(B x) { return enc(x); }
  __device__ static inline C cpiv(uint64_t code) { return (uint32_t)code; }
};

// Geometry of the partition pass per element type and pass type.
// KPT_ = 0: the default keys per thread of the key type; a workgroup of twice
// the threads with half the keys each (KPT_ = default / 2) has the same chunk.
template <int DT, bool HASV, bool TWO, int NT_ = (TWO ? kPartNT2 : kPartNT1), int KPT_ = 0> struct PartCfg {
  using B = typename Codec<DT>::B;
  static constexpr int NT = NT_;                                        // threads
  static constexpr int NW = NT / kWave;
  static constexpr int KB = (int)sizeof(B);
  static constexpr int VEC = 16 / KB;                                   // keys per 16-byte load
  static constexpr int KPT = KPT_ ? KPT_ : (KB == 4 ? (HASV ? 16 : 32) : (HASV ? 8 : 16));  // keys per thread
  static constexpr int NLOAD = KPT / VEC;
  static constexpr uint64_t CH = (uint64_t)NT * KPT;                    // keys per chunk
  static constexpr uint64_t LINE = 128 / KB;                            // keys per 128-byte line
  static_assert(KPT % VEC == 0 && NW <= kWave, "layout");
};


// ---- device tables -----------------------------------------------------------

// A part of a level.  Pivots are codes: piv[0] splits the part; piv[1] and
// piv[2] split its < and > sides (its children); piv[3..6] split the children's
// < and > sides (its grandchildren, in the order <<, <>, ><, >>).
//
// One-level pass (flags without kSegTwo): the part is split by piv[0] with a
// left and a right cursor (sizes unknown in advance); the keys of each side are
// also counted against that side's pivot (piv[1] / piv[2]), so the children
// enter the next level with the sizes of their own classes known.
// Two-level pass (kSegTwo): nlt / neq, the numbers of keys below / equal to
// piv[0], are known, so the < and > regions are placed exactly and each is split
// by its own pivot with two cursors in the same pass: two levels of the
// recursion per read and write of the keys; the four grandchildren are counted
// against piv[3..6] for the pass after.
constexpr uint32_t kSegInS = 1, kSegTwo = 2;
struct Seg {
  uint64_t off;              // first key
  uint64_t piv[7];
  uint32_t len;
  uint32_t chunk_begin;      // first chunk of this part in the level's chunk space
  uint32_t depth;            // recursion depth
  uint32_t dmax;             // depth limit of the array it came from
  uint32_t req;              // request (array) the part belongs to
  uint32_t flags;            // kSegInS: the keys are in S (else K); kSegTwo: two-level pass
  uint32_t nlt, neq;         // keys below / equal to piv[0] (two-level pass)
};

// Counters of a part (kCtrStride words, four 128-byte lines, one per reservation
// counter): [kCtrA] left | right cursor (one-level: < | >; two-level: << | <>),
// [kCtrE] keys equal to piv[0] (staged payloads), [kCtrB] two-level: >< | >>
// cursors, [kCtrE12] two-level: keys equal to piv[1] | to piv[2] (staged
// payloads), [kCtrLook..+3] look-ahead counts (below | equal << 32): one-level
// [+0] < side vs piv[1], [+1] > side vs piv[2]; two-level [+0..3] the four
// grandchildren vs piv[3..6].  Atomics to one line are serialised, and a chunk's
// reservations (two, four with payloads) lie on its critical path: on separate
// lines they proceed side by side, which counts in a pass over few large parts,
// whose chunks all reserve on the same lines (2^28 int32, level 1 = two parts:
// 0.60 -> 0.56 ms per pass; with payloads 1.9 -> 1.13 ms).
constexpr int kCtrA = 0, kCtrE = 16, kCtrB = 32, kCtrE12 = 48, kCtrLook = 4;

struct FinItem {             // work of the finish kernel (len 0 = empty slot)
  uint64_t off;              // small part: first key; band: first band slot
  uint64_t src;              // band: first staged payload in VE
  uint64_t pivot;            // band: encoded key of the band
  uint32_t len;
  uint32_t kind;             // bit 1: small part lives in S; bits 2..31: request
};

// ---- persistent schedule (tsqs_persist.hpp): tasks, parts and the queue ----
//
// Workgroups of one kernel take tasks from a ring in device memory: chunks of
// a part to partition, chunks of a part whose exact pivot is being selected
// (one radix digit per round), or a piece of a long equal band.  A part lives
// in a pool (TPart); the workgroup that finishes the last chunk of a part
// plans it (bands, small children sorted on the spot, new parts and their
// tasks).  A count of keys not yet final ends the kernel when it reaches zero.
constexpr uint32_t kSegSel = 4;            // flag: the part's exact pivot is being selected
enum : uint32_t { kTaskPart = 0, kTaskSelect = 1, kTaskBand = 2 };
struct Task { uint32_t kind, id, c0, c1; };   // chunks [c0, c1) of part id / band piece c0 of band id
struct TPart {
  Seg s;                     // s.chunk_begin = 0
  uint32_t nchunks;          // chunks of the current phase (partition or one select round)
  uint32_t done;             // chunks of the current phase finished
  uint32_t round;            // select: digits fixed so far
  uint32_t krem;             // select: rank sought among the keys that match prefix
  uint64_t prefix, mask;     // select: the fixed digits (codes)
  uint32_t hslot, pad;       // select: histogram slot
};
// control words of the queue, one 128-byte line each
enum { kQHead = 0, kQTail = 16, kQLeft = 32, kQAbort = 48, kQParts = 64, kQBands = 80, kQHist = 96,
       kQFin = 112, kQFinw = 128, kQWords = 144 };
struct PCtx {
  Task *task;                      // ring of tasks
  unsigned long long *seq;         // per ring slot: index + 1 once the task at that index is written
  unsigned long long *ctl;         // kQWords control words
  TPart *parts;                    // part pool (null: no persistent schedule)
  unsigned long long *pctr;        // counter lines of the pool's parts (kCtrStride words each)
  uint32_t *hist;                  // select histograms, 256 words per slot
  FinItem *bands;                  // long bands waiting for band tasks
  FinItem *sfin;                   // small parts left for k_finish_list: workgroup-sized ones
                                   // from the front, wave-sized ones from the back
  unsigned long long qmask;        // ring slots - 1 (a power of two - 1)
  uint32_t part_cap, hist_cap, band_cap, grid;   // grid: workgroups of the persistent kernel
  uint32_t sfin_cap, pad2;
  unsigned long long iter_cap;     // loop iterations of a workgroup before it gives up
};

struct RootRec {             // an array to sort, given by place instead of by offsets
  uint64_t off;
  uint32_t len;
  uint32_t req;
};

struct LevelCtl {
  unsigned long long packed; // parts << 40 | chunks of this level
  unsigned long long keys;   // keys in the parts of this level
  unsigned int nbig;         // chunks of bands longer than kBandChunk
  unsigned int pad0;
  unsigned long long pad1;
};

struct Ctx {
  void *K, *S;
  uint32_t *V, *VS, *VE;
  Seg *seg0, *seg1;
  unsigned long long *ctr0, *ctr1;   // per part, stride kCtrStride: [0] = L | G << 32, [1] = E
  FinItem *fin, *finw;               // small-part slots (4 per part): workgroup / wave sized
  FinItem *band;                     // band slots (3 per part)
  FinItem *big;                      // chunks of long bands (appended)
  LevelCtl *lvl;
  unsigned long long *stats;         // kStripes x kStatWords
  unsigned int *err;
  unsigned int *pre;                 // presortedness words of a single array, or null (check off)
  const uint64_t *roots;             // nroots+1 offsets, or null: one root [0, n)
  const RootRec *root_recs;          // or the roots one by one (then roots is ignored)
  unsigned long long *req_left;      // keys not yet final, per request (null: not tracked)
  volatile unsigned int *req_flag;   // host-visible: set to 1 when a request's count hits 0
  volatile unsigned int *done_ring;  // host-visible: request + 1 of each completion, in order
  unsigned int *done_pos;            // completions so far (next ring position)
  uint32_t done_cap;                 // ring entries
  uint32_t fin_roots_only;           // k_finish: only the roots' slots (no level parts yet)
  int root_level;                    // level whose parts and finish work the roots join
  uint32_t ring;                     // 1: level indices wrap around kMaxLevels
  uint64_t n;
  uint32_t nroots;
  uint32_t small_max;
  uint32_t wave_max;                 // small parts up to this padded size go to one wave
  uint32_t samples;
  uint32_t depth_factor;
  uint32_t pivot_mode;               // 0 sampled median, 1 exact minimum
  uint32_t jitter;                   // per-call sample shift
  uint32_t seg_cap;                  // part records per level; child slots are 4 * seg_cap
  uint32_t big_cap;
  uint32_t presort_roots;            // 1: k_init checks each root for order itself (batches)
  PCtx p;                            // persistent schedule (p.parts null: none)
  // debug shadows (null: off), 3 n words: [0, n) and [n, 2n) the depth + 1 of the
  // part whose pass last stored each slot of K and of S, [2n, 3n) 1 once a slot
  // of K holds its final key (a band or a small part)
  unsigned int *dbg;
};

// ---- wave helpers ------------------------------------------------------------

__device__ inline uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of m in lanes below this one
// wave mask of a predicate
__device__ inline unsigned long long wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
// base + number of set bits of m in lanes below this one
__device__ inline uint32_t mbcnt_from(unsigned long long m, uint32_t base) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, base));
}
__device__ inline uint32_t mbcnt(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline uint32_t shfl_xor_u32(uint32_t v, int m) { return (uint32_t)__shfl_xor((int)v, m); }
__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = shfl_xor_u32((uint32_t)v, m), hi = shfl_xor_u32((uint32_t)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint32_t shfl_u32(uint32_t v, int src) { return (uint32_t)__shfl((int)v, src); }
__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = shfl_u32((uint32_t)v, src), hi = shfl_u32((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}
template <typename U> __device__ inline U shfl_xor_any(U v, int m);
template <> __device__ inline uint32_t shfl_xor_any<uint32_t>(uint32_t v, int m) { return shfl_xor_u32(v, m); }
template <> __device__ inline uint64_t shfl_xor_any<uint64_t>(uint64_t v, int m) { return shfl_xor_u64(v, m); }
// v of lane 0
template <typename U> __device__ inline U shfl_first(U v) {
  if constexpr (sizeof(U) == 8) return (U)shfl_u64((uint64_t)v, 0);
  else return (U)shfl_u32((uint32_t)v, 0);
}
// v of the next lane (lane 63 keeps its own)
template <typename U> __device__ inline U shfl_any_down1(U v) {
  const uint32_t l = lane_id();
  const int src = (int)(l < 63u ? l + 1u : l);
  if constexpr (sizeof(U) == 8) return (U)shfl_u64((uint64_t)v, src);
  else return (U)shfl_u32((uint32_t)v, src);
}

// LDS ordering between the lanes of one wave (a wave-scope barrier).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ascending bitonic sort of one value per lane across the 64 lanes
template <typename U>
__device__ inline U wave_sort64(U v) {
  const uint32_t lane = lane_id();
  for (uint32_t k = 2; k <= 64; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      U o = shfl_xor_any<U>(v, (int)j);
      bool up = (lane & k) == 0;
      bool lower = (lane & j) == 0;
      U mn = v < o ? v : o, mx = v < o ? o : v;
      v = (lower == up) ? mn : mx;
    }
  }
  return v;
}

// inclusive prefix sum across the wave
__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = (uint32_t)__shfl_up((int)x, o);
    if (lane >= (uint32_t)o) x += t;
  }
  return x;
}

// ---- pivot choice (one wave) ---------------------------------------------------

// Median of S samples (S odd, <= 63) at evenly spaced positions of Y[off, off+len);
// interior samples (not the first, middle or last) are shifted toward the middle
// or away from it by a per-call amount of at most a quarter spacing (the paper's
// sample jitter against crafted inputs, SV.C).
template <int DT>
__device__ inline typename Codec<DT>::B wave_sample_pivot(const typename Codec<DT>::B *Y,
                                                          uint64_t off, uint32_t len,
                                                          uint32_t S, uint32_t jitter) {
  using B = typename Codec<DT>::B;
  const uint32_t lane = lane_id();
  B v = ~(B)0;
  if (lane < S) {
    const uint64_t span = (uint64_t)len - 1;
    uint64_t pos = (uint64_t)lane * span / (S - 1);
    const uint64_t h = span / (S - 1);
    const uint32_t half = S / 2;
    if (lane != 0 && lane != half && lane != S - 1 && h >= 4) {
      int64_t d = (int64_t)(((uint64_t)jitter * (h / 2)) >> 32) - (int64_t)(h / 4);
      pos = lane < half ? (uint64_t)((int64_t)pos + d) : (uint64_t)((int64_t)pos - d);
    }
    v = Codec<DT>::enc(Y[off + pos]);
  }
  v = wave_sort64<B>(v);
  if constexpr (sizeof(B) == 8) return shfl_u64(v, (int)(S / 2));
  else return shfl_u32(v, (int)(S / 2));
}

template <typename B>
__device__ inline B shfl_any(B v, int src) {
  if constexpr (sizeof(B) == 8) return shfl_u64(v, src);
  else return shfl_u32(v, src);
}

// Pivots of a part from one sorted sample (whole wave).  S samples of
// Y[off, off+len) as in wave_sample_pivot; with own = the part's own pivot
// (own_known) or the sample median, the children's pivots are the medians of
// the samples below / above own, and the grandchildren's the medians of the
// samples in the four ranges those cut (a side without samples reuses the
// pivot that bounds it: the split then makes no progress there, and the depth
// limit bounds how often that can happen).  piv[0] = own.
template <int DT>
__device__ inline void wave_part_pivots(const typename Codec<DT>::B *Y, uint64_t off, uint32_t len,
                                        uint32_t S, uint32_t jitter, bool own_known,
                                        typename Codec<DT>::B own, uint64_t piv[7]) {
  using B = typename Codec<DT>::B;
  const uint32_t lane = lane_id();
  B v = ~(B)0;
  if (lane < S) {
    const uint64_t span = (uint64_t)len - 1;
    uint64_t pos = (uint64_t)lane * span / (S - 1);
    const uint64_t h = span / (S - 1);
    const uint32_t half = S / 2;
    if (lane != 0 && lane != half && lane != S - 1 && h >= 4) {
      int64_t dd = (int64_t)(((uint64_t)jitter * (h / 2)) >> 32) - (int64_t)(h / 4);
      pos = lane < half ? (uint64_t)((int64_t)pos + dd) : (uint64_t)((int64_t)pos - dd);
    }
    v = Codec<DT>::enc(Y[off + pos]);
  }
  v = wave_sort64<B>(v);
  const bool in = lane < S;
  if (!own_known) own = shfl_any<B>(v, (int)(S / 2));
  // samples below / not above a value: the sorted prefix lengths
  auto below = [&](B x) { return (uint32_t)__popcll(__ballot(in && v < x)); };
  auto upto = [&](B x) { return (uint32_t)__popcll(__ballot(in && v <= x)); };
  auto med = [&](uint32_t lo, uint32_t hi, B dflt) {   // median of samples [lo, hi)
    return hi > lo ? shfl_any<B>(v, (int)(lo + (hi - lo - 1) / 2)) : dflt;
  };
  const uint32_t a = below(own), b = upto(own);
  const B pl = med(0, a, own), pg = med(b, S, own);
  const uint32_t a1 = below(pl), b1 = upto(pl), a2 = below(pg), b2 = upto(pg);
  piv[0] = (uint64_t)own;
  piv[1] = (uint64_t)pl;
  piv[2] = (uint64_t)pg;
  piv[3] = (uint64_t)med(0, a1 < a ? a1 : a, pl);
  piv[4] = (uint64_t)med(b1 < a ? b1 : a, a, pl);
  piv[5] = (uint64_t)med(b, a2 > b ? a2 : b, pg);
  piv[6] = (uint64_t)med(b2 > b ? b2 : b, S, pg);
}

// Exact k-th smallest code of Y[off, off+len) by most-significant-digit radix
// select (8-bit digits, a 256-bin LDS histogram per wave).  Read-only.
template <int DT>
__device__ typename Codec<DT>::B wave_select(const typename Codec<DT>::B *Y, uint64_t off,
                                             uint32_t len, uint32_t k, uint32_t *hist) {
  using B = typename Codec<DT>::B;
  constexpr int BITS = (int)sizeof(B) * 8;
  const uint32_t lane = lane_id();
  B prefix = 0, mask = 0;
  uint32_t krem = k;
  for (int shift = BITS - 8; shift >= 0; shift -= 8) {
    for (int i = 0; i < 4; i++) hist[lane * 4 + i] = 0;
    wave_lds_sync();
    for (uint32_t i = lane; i < len; i += kWave) {
      const B u = Codec<DT>::enc(Y[off + i]);
      if ((u & mask) == prefix) atomicAdd(&hist[(uint32_t)(u >> shift) & 255u], 1u);
    }
    wave_lds_sync();
    uint32_t h[4], s = 0;
    for (int i = 0; i < 4; i++) { h[i] = hist[lane * 4 + i]; s += h[i]; }
    const uint32_t incl = wave_incl_scan(s);
    const uint32_t excl = incl - s;
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
    krem -= below;
    prefix |= (B)dig << shift;
    mask |= (B)255 << shift;
    wave_lds_sync();
  }
  return prefix;
}


// ---- emission ---------------------------------------------------------------------

__device__ inline uint32_t next_pow2(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Number of chunks of a part [off, off+len) of a buffer: the part's chunks are
// consecutive windows of CH keys (of its pass type) from the 128-byte line
// holding its first key (so a part of up to CH keys, less its offset in that
// line, is one chunk, and every wave's loads cover whole lines).
template <int DT, bool HASV>
__device__ inline uint32_t part_chunks(const void *buf, uint64_t off, uint32_t len, bool two) {
  using C1 = PartCfg<DT, HASV, false>;
  using C2 = PartCfg<DT, HASV, true>;
  const uint64_t a0 = (uint64_t)(uintptr_t)buf / C1::KB + off;
  const uint64_t ch = two ? C2::CH : C1::CH;
  return (uint32_t)((a0 % C1::LINE + len + ch - 1) / ch);
}


__device__ inline void stat_add(const Ctx &c, int which, unsigned long long v) {
  if (v) atomicAdd(&c.stats[(size_t)(blockIdx.x % kStripes) * kStatWords + which], v);
}

// Index of the level after d (with ring, indices wrap; without, kMaxLevels is
// out of range and reported as an error where it is used).
__device__ inline int level_after(const Ctx &c, int d) {
  return d + 1 < kMaxLevels ? d + 1 : (c.ring ? 0 : kMaxLevels);
}

// n keys of request req are final (one thread; the caller has made its stores
// visible at device scope).  The thread that brings the count to zero raises the
// request's host-visible flag and appends the request to the completion ring.
__device__ inline void req_final(const Ctx &c, uint32_t req, uint32_t n) {
  if (n == 0) return;
  const unsigned long long old = atomicSub(&c.req_left[req], (unsigned long long)n);
  if (old == (unsigned long long)n) {
    __threadfence_system();
    c.req_flag[req] = 1u;
    const unsigned int p = atomicAdd(c.done_pos, 1u);
    c.done_ring[p % c.done_cap] = req + 1u;
  }
}

// Debug shadows.  A part's pass stores each slot of its range (in the other
// buffer) once: a slot that already holds this part's stamp was reserved twice.
// The stamp is the part's depth + 1; a slot lies in one part per depth, so the
// stamps of earlier passes never match.
__device__ inline void dbg_store(const Ctx &c, bool to_k, uint64_t i, uint32_t depth) {
  const uint32_t old = atomicExch(&c.dbg[(to_k ? 0ull : c.n) + i], depth + 1u);
  if (old == depth + 1u) atomicOr(c.err, kErrShadow);
  if (to_k && c.dbg[2ull * c.n + i] != 0u) atomicOr(c.err, kErrShadow);   // over a final slot
}
// A slot of K receives its final key (band fill, small part, a part of one key).
__device__ inline void dbg_final(const Ctx &c, uint64_t i) {
  if (atomicExch(&c.dbg[2ull * c.n + i], 1u) != 0u) atomicOr(c.err, kErrShadow);
}
// Writes the small-part item of a child into its fixed slot of the wave or the
// workgroup array and an empty item into the other (one lane).  A single key
// already in K needs no work and is final at once.
__device__ inline void put_small(const Ctx &c, uint32_t slot, uint64_t off, uint32_t len, bool in_s,
                                 uint32_t req) {
  const bool real = len > 1 || (len == 1 && in_s);
  const bool wave = next_pow2(len) <= c.wave_max;
  FinItem it;
  it.off = off; it.src = 0; it.pivot = 0; it.kind = (in_s ? 2u : 0u) | (req << 2);
  it.len = (real && wave) ? len : 0u;
  c.finw[slot] = it;
  it.len = (real && !wave) ? len : 0u;
  c.fin[slot] = it;
  if (!real && len == 1 && c.req_left) req_final(c, req, 1u);
  if (!real && len == 1 && c.dbg) dbg_final(c, off);
}

// Band of a part: short bands go to the part's band slot, long ones are cut
// into kBandChunk pieces appended to the long-band list (one lane).
__device__ inline void put_band(const Ctx &c, int level, uint32_t si, uint64_t off, uint64_t src,
                                uint32_t len, uint64_t pivot, uint32_t req) {
  FinItem it;
  it.off = off; it.src = src; it.pivot = pivot; it.len = len <= kBandChunk ? len : 0u;
  it.kind = req << 2;
  c.band[si] = it;
  if (len <= kBandChunk) return;
  const uint32_t nch = (len + kBandChunk - 1) / kBandChunk;
  const uint32_t i0 = atomicAdd(&c.lvl[level].nbig, nch);
  if (i0 + nch > c.big_cap) { atomicOr(c.err, kErrFinCap); return; }
  for (uint32_t q = 0; q < nch; q++) {
    const uint32_t base = q * kBandChunk;
    it.off = off + base; it.src = src + base;
    it.len = (len - base < kBandChunk) ? (len - base) : kBandChunk;
    c.big[i0 + q] = it;
  }
}

// ---- persistent schedule: ring, pool, grid-wide selection ----------------------

__device__ inline void persist_abort(const Ctx &c, uint32_t why) {
  atomicOr(c.err, why);
  __hip_atomic_store(&c.p.ctl[kQAbort], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes n tasks, task i built by make(i) (whole wave; lane 0 reserves the
// ring slots).  What the wave wrote before is visible to the workgroups that
// take them.  False (and the run aborted) if the ring would overrun slots not
// yet read.
template <typename F>
__device__ inline bool push_tasks(const Ctx &c, uint32_t n, F make) {
  if (n == 0) return true;
  const uint32_t lane = lane_id();
  unsigned long long base = 0;
  uint32_t ok = 1;
  if (lane == 0) {
    base = atomicAdd(&c.p.ctl[kQTail], (unsigned long long)n);
    const unsigned long long head =
        __hip_atomic_load(&c.p.ctl[kQHead], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // slots are reused once read: keep one claim per workgroup of margin
    if (base + n > head + (c.p.qmask + 1) - 2ull * c.p.grid) ok = 0;
  }
  ok = shfl_u32(ok, 0);
  base = shfl_u64(base, 0);
  if (!ok) {
    if (lane == 0) persist_abort(c, kErrQueue);
    return false;
  }
  __threadfence();
  for (uint32_t i = lane; i < n; i += kWave) c.p.task[(base + i) & c.p.qmask] = make(i);
  __threadfence();
  for (uint32_t i = lane; i < n; i += kWave)
    __hip_atomic_store(&c.p.seq[(base + i) & c.p.qmask], base + i + 1, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Chunks of a pool part's partition pass (persistent workgroups of kPNT
// threads): windows of CH keys from the 128-byte line of its first key.
template <int DT, bool HASV>
__device__ inline uint32_t pool_chunks(const Ctx &c, uint64_t off, uint32_t len, uint32_t flags) {
  using C1 = PartCfg<DT, HASV, false, kPNT>;
  using C2 = PartCfg<DT, HASV, true, kPNT>;
  const void *buf = (flags & kSegInS) ? c.S : c.K;
  const uint64_t a0 = (uint64_t)(uintptr_t)buf / C1::KB + off;
  const uint64_t ch = (flags & kSegTwo) ? C2::CH : C1::CH;
  return (uint32_t)((a0 % C1::LINE + len + ch - 1) / ch);
}

// Writes pool part id (lane 0 writes the record; lanes clear its counters).
__device__ inline void pool_put(const Ctx &c, uint32_t id, const TPart &tp) {
  const uint32_t lane = lane_id();
  if (lane == 0) c.p.parts[id] = tp;
  if (lane < (uint32_t)kCtrStride) c.p.pctr[(size_t)id * kCtrStride + lane] = 0ull;
}

// Tasks of a pool part's current phase (partition or one select round).
__device__ inline bool pool_tasks(const Ctx &c, uint32_t id, uint32_t kind, uint32_t nchunks) {
  return push_tasks(c, (nchunks + kTaskChunks - 1) / kTaskChunks, [&](uint32_t i) {
    Task t;
    t.kind = kind; t.id = id; t.c0 = i * kTaskChunks;
    t.c1 = (i + 1) * kTaskChunks < nchunks ? (i + 1) * kTaskChunks : nchunks;
    return t;
  });
}

// The grid-wide selection of the k-th smallest key of a part, its exact pivot
// (the depth limit, or the exact-minimum test mode): a pool part in select
// phase and its first round of tasks.  Whole wave.  False if no histogram
// slot or pool part is free (the caller then selects with one wave).  With
// count, the part's keys are added to the count of keys not yet final (a part
// that no pool part held before).
__device__ inline bool start_select(const Ctx &c, uint64_t off, uint32_t len, uint32_t depth,
                                    uint32_t dmax, uint32_t req, bool in_s, uint32_t k, bool count) {
  const uint32_t lane = lane_id();
  uint32_t id = ~0u, slot = ~0u;
  if (lane == 0) {
    const unsigned long long hs = atomicAdd(&c.p.ctl[kQHist], 1ull);
    if (hs < c.p.hist_cap) {
      const unsigned long long pid = atomicAdd(&c.p.ctl[kQParts], 1ull);
      if (pid < c.p.part_cap) { id = (uint32_t)pid; slot = (uint32_t)hs; }
    }
  }
  id = shfl_u32(id, 0);
  slot = shfl_u32(slot, 0);
  if (id == ~0u) return false;
  TPart tp;
  tp.s.off = off;
#pragma unroll
  for (int q = 0; q < 7; q++) tp.s.piv[q] = 0;
  tp.s.len = len; tp.s.chunk_begin = 0; tp.s.depth = depth; tp.s.dmax = dmax; tp.s.req = req;
  tp.s.flags = (in_s ? kSegInS : 0u) | kSegSel;
  tp.s.nlt = 0; tp.s.neq = 0;
  tp.nchunks = (len + kSelChunk - 1) / kSelChunk;
  tp.done = 0; tp.round = 0; tp.krem = k; tp.prefix = 0; tp.mask = 0;
  tp.hslot = slot; tp.pad = 0;
  pool_put(c, id, tp);
  for (uint32_t q = lane; q < 256; q += kWave) c.p.hist[(size_t)slot * 256 + q] = 0u;
  if (count && lane == 0) atomicAdd(&c.p.ctl[kQLeft], (unsigned long long)len);
  pool_tasks(c, id, kTaskSelect, tp.nchunks);
  return true;
}

// Parts a workgroup emits in one iteration (up to 4 per wave), staged in LDS
// and reserved in the next level with a single atomic (records keep the wave
// order, so chunk_begin stays increasing with the record index).
constexpr int kPendPerWave = 4;
struct PendLds {
  Seg rec[kPlanNW][kPendPerWave];
  uint32_t n[kPlanNW], ch[kPlanNW];
  unsigned long long keys[kPlanNW], old;
};

// A child part of `len` keys at Y[off, ...) (Y = S if in_s, else K), depth
// `depth`.  Small: its finish slot.  Large: its pivots and pass type, staged in
// pend (lane 0).  With own_known, own is the pivot the child already has and
// nlt / neq the counts of its keys below / equal to it (look-ahead of the pass
// that produced it): the child gets a two-level pass.  Otherwise (payloads, the
// depth limit, the exact-minimum test mode, or a root) it gets a one-level pass
// around the sample median, or around the exact median / minimum found by radix
// select.  Whole wave.
// Depth a child part enters with: its parent's depth plus the recursion levels
// between them, or the depth limit itself when the child kept more than 15/16
// of the parent's keys.  A split that unbalanced sends the child and its whole
// subtree to exact-median pivots at once, rather than after the up to
// 2 ceil(log2 n) nearly full passes the depth limit alone allows.  A median of
// up to 63 jittered samples practically never splits that badly unless the
// input is built against the sampling.
__device__ inline uint32_t child_depth(uint32_t pdepth, uint32_t levels, uint32_t plen, uint32_t clen,
                                       uint32_t dmax) {
  const uint32_t d = pdepth + levels;
  return (d < dmax && (uint64_t)clen * 16 > (uint64_t)plen * 15) ? dmax : d;
}

template <int DT, bool HASV>
__device__ inline void child(const Ctx &c, uint32_t slot, uint64_t off, uint32_t len, uint32_t depth,
                             uint32_t dmax, uint32_t req, bool in_s, bool own_known, uint64_t own,
                             uint32_t nlt, uint32_t neq, uint32_t *hist, PendLds &pend, uint32_t wv,
                             unsigned long long &small_parts, unsigned long long &small_keys) {
  using B = typename Codec<DT>::B;
  const uint32_t lane = lane_id();
  if (len <= c.small_max) {
    if (lane == 0) {
      put_small(c, slot, off, len, in_s, req);
      if (len > 1 || (len == 1 && in_s)) { small_parts++; small_keys += len; }
    }
    return;
  }
  const B *Y = (const B *)(in_s ? c.S : c.K);
  uint32_t S = c.samples;
  if (S > len) S = (len & 1) ? len : len - 1;
  const bool exact = c.pivot_mode == 1 || depth >= dmax;
  const bool fits = (uint64_t)nlt + neq <= len;
  if (own_known && !fits && lane == 0) atomicOr(c.err, kErrCount);
  const bool two = own_known && !exact && fits;
  B p0 = (B)own;
  if (exact) {
    const uint32_t k = (c.pivot_mode == 1 && depth < dmax) ? 0u : len / 2;
    if (lane == 0 && depth >= dmax) stat_add(c, kStFallback, 1ull);
    // a large part: its exact pivot is selected by the whole grid of the
    // persistent schedule (the part waits there); else by this wave
    if (len > kSelInline && c.p.parts &&
        start_select(c, off, len, depth, dmax, req, in_s, k, true)) {
      if (lane == 0) put_small(c, slot, 0, 0, false, req);
      return;
    }
    p0 = wave_select<DT>(Y, off, len, k, hist);
  }
  uint64_t piv[7];
  wave_part_pivots<DT>(Y, off, len, S, c.jitter, exact || two, p0, piv);
  if (lane == 0) {
    put_small(c, slot, 0, 0, false, req);
    const uint32_t i = pend.n[wv];
    Seg &r = pend.rec[wv][i];
    r.off = off;
#pragma unroll
    for (int k = 0; k < 7; k++) r.piv[k] = piv[k];
    r.len = len;
    r.chunk_begin = part_chunks<DT, HASV>(in_s ? c.S : c.K, off, len, two);   // chunks, until flushed
    r.depth = depth;
    r.dmax = dmax;
    r.req = req;
    r.flags = (in_s ? kSegInS : 0u) | (two ? kSegTwo : 0u);
    r.nlt = two ? nlt : 0u;
    r.neq = two ? neq : 0u;
    pend.n[wv] = i + 1;
    pend.ch[wv] += r.chunk_begin;
    pend.keys[wv] += len;
  }
}

// Reserve the workgroup's staged parts in level lvl_next with one atomic and
// write them out (whole workgroup; clears the staging area).
template <int DT, bool HASV>
__device__ inline void flush_parts(const Ctx &c, int lvl_next, PendLds &pend) {
  const uint32_t wv = threadIdx.x / kWave, lane = threadIdx.x & 63u;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tp = 0, tc = 0;
    unsigned long long tk = 0;
    for (int i = 0; i < kPlanNW; i++) { tp += pend.n[i]; tc += pend.ch[i]; tk += pend.keys[i]; }
    pend.old = 0;
    if (tp > 0) {
      if (lvl_next >= kMaxLevels) {
        atomicOr(c.err, kErrLevel);
        pend.old = ~0ull;
      } else {
        pend.old = atomicAdd(&c.lvl[lvl_next].packed, ((unsigned long long)tp << 40) | tc);
        atomicAdd(&c.lvl[lvl_next].keys, tk);
      }
    }
  }
  __syncthreads();
  if (lane == 0 && pend.n[wv] > 0 && pend.old != ~0ull) {
    uint32_t idx = (uint32_t)(pend.old >> 40), cb = (uint32_t)(pend.old & kTileMask);
    for (uint32_t i = 0; i < wv; i++) { idx += pend.n[i]; cb += pend.ch[i]; }
    Seg *segs = (lvl_next & 1) ? c.seg1 : c.seg0;
    unsigned long long *ctr = (lvl_next & 1) ? c.ctr1 : c.ctr0;
    for (uint32_t q = 0; q < pend.n[wv]; q++, idx++) {
      if (idx >= c.seg_cap) { atomicOr(c.err, kErrSegCap); break; }
      Seg r = pend.rec[wv][q];
      const uint32_t nch = r.chunk_begin;
      r.chunk_begin = cb;
      segs[idx] = r;
      unsigned long long *cp = ctr + (size_t)idx * kCtrStride;
      cp[kCtrA] = 0ull;
      cp[kCtrE] = 0ull;
      cp[kCtrB] = 0ull;
      cp[kCtrE12] = 0ull;
#pragma unroll
      for (int k = 0; k < 4; k++) cp[kCtrLook + k] = 0ull;
      cb += nch;
    }
  }
  __syncthreads();
  if (lane == 0) { pend.n[wv] = 0; pend.ch[wv] = 0; pend.keys[wv] = 0; }
  __syncthreads();
}

// ---- kernels ------------------------------------------------------------------------

static __global__ void k_reset(Ctx c) {
  for (int i = threadIdx.x; i < kMaxLevels; i += blockDim.x) {
    c.lvl[i].packed = 0ull; c.lvl[i].keys = 0ull; c.lvl[i].nbig = 0u;
  }
  for (int i = threadIdx.x; i < kStripes * kStatWords; i += blockDim.x) c.stats[i] = 0ull;
  if (threadIdx.x == 0) *c.err = 0u;
  if (c.pre && threadIdx.x < 2) c.pre[threadIdx.x] = 0u;
  if (c.p.ctl && threadIdx.x == 0) {
    // ring indices only grow (a slot's sequence word then never matches an
    // index of an earlier call); the other control words start at zero
    unsigned long long *q = c.p.ctl;
    const unsigned long long m = q[kQHead] > q[kQTail] ? q[kQHead] : q[kQTail];
    q[kQHead] = m; q[kQTail] = m;
    q[kQLeft] = 0; q[kQAbort] = 0; q[kQParts] = 0; q[kQBands] = 0; q[kQHist] = 0;
    q[kQFin] = 0; q[kQFinw] = 0;
  }
}

// Clears n words (setup of a fixed ring; no memset nodes in captured work).
static __global__ void k_dbg_clear(Ctx c) {
  const uint64_t m = 3ull * c.n, st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += st) c.dbg[i] = 0u;
}
// Test modes of the shadows (TSQS_OPT_DEBUG 2, 3): one entry planted before the
// sort, as if a slot had been finalised already (2: slot 0 of K) or stored by
// the root's pass already (3: slot 0 of S, the stamp of depth 0), so that a
// correct sort must report a shadow error.
static __global__ void k_dbg_plant(Ctx c, int mode) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (mode == 2) c.dbg[2ull * c.n] = 1u;
    else c.dbg[c.n] = 1u;
  }
}
// After the sort: every slot of K holds its final key.
static __global__ void k_dbg_end(Ctx c) {
  const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.n; i += st)
    bad |= c.dbg[2ull * c.n + i] == 0u;
  if (bad) atomicOr(c.err, kErrShadow);
}

static __global__ void k_zero(unsigned long long *p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Clears the counters of level `lvl` (a serving tick reuses level indices
// around a ring; the counters of the next level must start at zero).
static __global__ void k_level_clear(Ctx c, int lvl) {
  if (threadIdx.x == 0) {
    c.lvl[lvl].packed = 0ull; c.lvl[lvl].keys = 0ull; c.lvl[lvl].nbig = 0u;
  }
}

// ---- presortedness check (SIII.I) -------------------------------------------------
//
// The paper guesses a possibly sorted or possibly reversed part from the order of
// its pivot samples and then runs a handler that either confirms the guess or
// falls back to the partition.  For a single array this is done before the first
// pass: pre[0] is the guess from 64 evenly spaced keys (first and last included):
// 1 = non-decreasing, 2 = non-increasing, 0 = neither; pre[1] is set when a scan
// of every adjacent pair finds one against the guess.  A confirmed
// non-increasing array is reversed in place (keys and payloads), and a confirmed
// array then needs no pass at all.  Both words are cleared by k_reset.
__device__ inline bool presorted(const Ctx &c) {
  return c.pre != nullptr && c.pre[0] != 0u && c.pre[1] == 0u;
}

constexpr int kPreNT = 256;       // threads of the presortedness kernels
// Largest array of a batch that its wave checks (one wave streams it; a larger
// array would hold every later level behind it).
constexpr uint32_t kPresortRootMax = 1u << 16;
constexpr int kPreRows = 16;      // keys per thread per chunk (one row = kPreNT keys)

template <int DT>
__global__ __launch_bounds__(kPreNT) void k_presort_scan(Ctx c) {
  using B = typename Codec<DT>::B;
  using Cm = typename Codec<DT>::C;
  const B *K = (const B *)c.K;
  const uint64_t n = c.n;
  const uint32_t lane = threadIdx.x & 63u;
  // the guess (every wave takes the same one): 64 evenly spaced keys in
  // non-decreasing or in non-increasing order
  uint32_t mode;
  {
    const uint64_t pos = (uint64_t)lane * (n - 1) / (kWave - 1);
    const B x = K[pos];
    const B z = shfl_any_down1<B>(x);          // x of the next lane (lane 63: itself)
    const Cm a = Codec<DT>::ckey(x), b = Codec<DT>::ckey(z);
    const bool up = wave_ballot(a > b) == 0ull, down = wave_ballot(a < b) == 0ull;
    mode = up ? 1u : (down ? 2u : 0u);
    if (blockIdx.x == 0 && threadIdx.x == 0) c.pre[0] = mode;
    if (mode == 0u) return;
  }
  // every adjacent pair, one wave per step of kWave * kPreRows keys (rows of kWave
  // consecutive keys; the pair that leaves a row is closed by the next row's lane 0)
  const uint64_t wkeys = (uint64_t)kWave * kPreRows;
  const uint64_t steps = (n + wkeys - 1) / wkeys;
  const uint64_t nw = (uint64_t)gridDim.x * (kPreNT / kWave);
  for (uint64_t st = (uint64_t)blockIdx.x * (kPreNT / kWave) + threadIdx.x / kWave; st < steps; st += nw) {
    const uint32_t stop = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&c.pre[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (stop) return;
    const uint64_t base = st * wkeys;
    B x[kPreRows];
#pragma unroll
    for (int r = 0; r < kPreRows; r++) {
      const uint64_t i = base + (uint64_t)r * kWave + lane;
      x[r] = i < n ? K[i] : B(0);
    }
    const B after = base + wkeys < n ? K[base + wkeys] : B(0);
    bool bad = false;
#pragma unroll
    for (int r = 0; r < kPreRows; r++) {
      const uint64_t i = base + (uint64_t)r * kWave + lane;
      B nb = shfl_any_down1<B>(x[r]);
      const B first_next = r + 1 < kPreRows ? shfl_first<B>(x[r + 1 < kPreRows ? r + 1 : r]) : after;
      if (lane == 63u) nb = first_next;
      if (i + 1 < n) {
        const Cm a = Codec<DT>::ckey(x[r]), b = Codec<DT>::ckey(nb);
        bad |= mode == 1u ? a > b : a < b;
      }
    }
    if (wave_ballot(bad) != 0ull && lane == 0) atomicOr(&c.pre[1], 1u);
  }
}

// Reverses a confirmed non-increasing array (and its payloads) in place.
template <int DT, bool HASV>
__global__ __launch_bounds__(kPreNT) void k_presort_reverse(Ctx c) {
  using B = typename Codec<DT>::B;
  if (c.pre[0] != 2u || c.pre[1] != 0u) return;
  B *K = (B *)c.K;
  const uint64_t n = c.n, half = n / 2;
  const uint64_t step = (uint64_t)gridDim.x * kPreNT;
  for (uint64_t i = (uint64_t)blockIdx.x * kPreNT + threadIdx.x; i < half; i += step) {
    const uint64_t j = n - 1 - i;
    const B a = K[i], b = K[j];
    K[i] = b; K[j] = a;
    if (HASV) {
      const uint32_t va = c.V[i], vb = c.V[j];
      c.V[i] = vb; c.V[j] = va;
    }
  }
}

// The same check for one root by one wave (batches: many arrays, one wave each):
// the 64-key guess, then every adjacent pair until one is against it; a
// non-increasing root is reversed in place.  Returns 0, 1 (non-decreasing) or 2
// (was non-increasing, now reversed).
template <int DT, bool HASV>
__device__ inline uint32_t wave_presort_root(const Ctx &c, uint64_t off, uint32_t len) {
  using B = typename Codec<DT>::B;
  using Cm = typename Codec<DT>::C;
  B *K = (B *)c.K + off;
  const uint32_t lane = lane_id();
  uint32_t mode;
  {
    const uint32_t pos = (uint32_t)((uint64_t)lane * (len - 1) / (kWave - 1));
    const B x = K[pos];
    const B z = shfl_any_down1<B>(x);
    const Cm a = Codec<DT>::ckey(x), b = Codec<DT>::ckey(z);
    const bool up = wave_ballot(a > b) == 0ull, down = wave_ballot(a < b) == 0ull;
    mode = up ? 1u : (down ? 2u : 0u);
  }
  if (mode == 0u) return 0u;
  const uint32_t wkeys = (uint32_t)kWave * kPreRows;
  for (uint32_t base = 0; base < len; base += wkeys) {
    B x[kPreRows];
#pragma unroll
    for (int r = 0; r < kPreRows; r++) {
      const uint32_t i = base + (uint32_t)r * kWave + lane;
      x[r] = i < len ? K[i] : B(0);
    }
    const B after = base + wkeys < len ? K[base + wkeys] : B(0);
    bool bad = false;
#pragma unroll
    for (int r = 0; r < kPreRows; r++) {
      const uint32_t i = base + (uint32_t)r * kWave + lane;
      B nb = shfl_any_down1<B>(x[r]);
      const B first_next = r + 1 < kPreRows ? shfl_first<B>(x[r + 1 < kPreRows ? r + 1 : r]) : after;
      if (lane == 63u) nb = first_next;
      if (i + 1 < len) {
        const Cm a = Codec<DT>::ckey(x[r]), b = Codec<DT>::ckey(nb);
        bad |= mode == 1u ? a > b : a < b;
      }
    }
    if (wave_ballot(bad) != 0ull) return 0u;
  }
  if (mode == 2u) {
    // kRevU pairs per lane in flight: all loads of a step before its stores
    constexpr int kRevU = 8;
    const uint32_t half = len / 2;
    for (uint32_t i0 = 0; i0 < half; i0 += kWave * kRevU) {
      B a[kRevU], b[kRevU];
#pragma unroll
      for (int u = 0; u < kRevU; u++) {
        const uint32_t i = i0 + (uint32_t)u * kWave + lane;
        if (i < half) { a[u] = K[i]; b[u] = K[len - 1 - i]; }
      }
#pragma unroll
      for (int u = 0; u < kRevU; u++) {
        const uint32_t i = i0 + (uint32_t)u * kWave + lane;
        if (i < half) { K[i] = b[u]; K[len - 1 - i] = a[u]; }
      }
      if (HASV) {
        uint32_t *V = c.V + off;
        uint32_t va[kRevU], vb[kRevU];
#pragma unroll
        for (int u = 0; u < kRevU; u++) {
          const uint32_t i = i0 + (uint32_t)u * kWave + lane;
          if (i < half) { va[u] = V[i]; vb[u] = V[len - 1 - i]; }
        }
#pragma unroll
        for (int u = 0; u < kRevU; u++) {
          const uint32_t i = i0 + (uint32_t)u * kWave + lane;
          if (i < half) { V[i] = vb[u]; V[len - 1 - i] = va[u]; }
        }
      }
    }
  }
  return mode;
}

// Roots: one wave per array (workgroup-uniform iterations).  A root is depth 0,
// lives in K, gets a one-level pass, and its small-part slot is 4 * seg_cap +
// root index.
template <int DT, bool HASV>
__global__ __launch_bounds__(kPlanNT) void k_init(Ctx c) {
  __shared__ uint32_t hist[kPlanNW][256];
  __shared__ PendLds pend;
  const uint32_t wv = threadIdx.x / kWave;
  if ((threadIdx.x & 63u) == 0) { pend.n[wv] = 0; pend.ch[wv] = 0; pend.keys[wv] = 0; }
  __syncthreads();
  unsigned long long small_parts = 0, small_keys = 0;
  for (uint32_t base = blockIdx.x * kPlanNW; base < c.nroots; base += gridDim.x * kPlanNW) {
    const uint32_t j = base + wv;
    if (j < c.nroots) {
      uint64_t off;
      uint32_t len, req = 0;
      if (c.root_recs) {
        const RootRec r = c.root_recs[j];
        off = r.off; len = r.len; req = r.req;
        if (c.req_left && lane_id() == 0) c.req_left[req] = len;
      } else {
        off = c.roots ? c.roots[j] : 0ull;
        len = (uint32_t)((c.roots ? c.roots[j + 1] : c.n) - off);
      }
      uint32_t lg = 0;
      while (lg < 32 && (1ull << lg) < (unsigned long long)len) lg++;
      if (presorted(c)) {
        // already in order (or reversed into order): no pass and no finish work
        if (lane_id() == 0) {
          put_small(c, 4 * c.seg_cap + j, off, 0u, false, req);
          stat_add(c, kStPresorted, (unsigned long long)c.pre[0]);
        }
      } else if (c.presort_roots && len > c.small_max && len <= kPresortRootMax &&
                 wave_presort_root<DT, HASV>(c, off, len) != 0u) {
        if (lane_id() == 0) {
          put_small(c, 4 * c.seg_cap + j, off, 0u, false, req);
          stat_add(c, kStPresortedRoots, 1ull);
        }
      } else
      child<DT, HASV>(c, 4 * c.seg_cap + j, off, len, 0u, c.depth_factor * lg, req, false, false, 0ull,
                      0u, 0u, hist[wv], pend, wv, small_parts, small_keys);
    }
    flush_parts<DT, HASV>(c, c.root_level, pend);
  }
  if ((threadIdx.x & 63u) == 0) {
    stat_add(c, kStSmallParts, small_parts);
    stat_add(c, kStSmallKeys, small_keys);
  }
}

// v := x in lane L of v; the other lanes keep their value
template <int L>
__device__ inline void lane_put(uint32_t &v, uint32_t x) {
  asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "n"(L));
}
// f(integral_constant<int, I>) for I = B .. E-1, expanded at compile time
template <int B, int E, typename F>
__device__ __attribute__((always_inline)) inline void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
// hide a value's origin from the optimiser (no instruction is emitted)
template <typename T>
__device__ inline void opaque_v(T &x) { asm volatile("" : "+v"(x)); }
template <typename T>
__device__ inline void opaque_s(T &x) { asm volatile("" : "+s"(x)); }

// c ? a : b on values (a conditional on lvalues would select their addresses,
// which keeps the variables out of registers)
template <typename T>
__device__ __attribute__((always_inline)) inline T pick(bool c, T a, T b) { return c ? a : b; }

// &base[i]; unless WIDE, i * sizeof(T) must fit in 32 bits (the address is
// then formed as a uniform base plus a 32-bit lane offset)
// partition passes that stage the next chunk's keys through LDS
constexpr bool kStageOne = true, kStageTwo = false;

// a part record in the constant address space
using CSeg = __attribute__((address_space(4))) Seg;
__device__ inline Seg load_seg(const CSeg *p) {
  Seg r;
  r.off = p->off;
#pragma unroll
  for (int k = 0; k < 7; k++) r.piv[k] = p->piv[k];
  r.len = p->len; r.chunk_begin = p->chunk_begin; r.depth = p->depth; r.dmax = p->dmax;
  r.req = p->req; r.flags = p->flags; r.nlt = p->nlt; r.neq = p->neq;
  return r;
}

// a part record written during the same kernel (the persistent schedule):
// ordinary global loads
__device__ inline Seg load_seg(const Seg *p) { return *p; }

// s_waitcnt immediate (gfx9 encoding): lgkmcnt(0), the other counters free
constexpr int kWaitLgkm0 = 0xC07F;

template <bool WIDE, typename T>
__device__ inline T *at(T *base, uint32_t i) {
  if constexpr (WIDE) return base + i;
  else return (T *)((char *)base + (uint32_t)(i * (uint32_t)sizeof(T)));
}

// LDS of a partition workgroup: per-wave class counts (one-level [<, >,
// look-ahead <<, <=, ><, >=, = (payloads)], two-level [<<, <>, ><, >>, = of
// each pivot (payloads), then the look-ahead sums as packed 16-bit fields]),
// the part of the first chunk, and the stage: the keys of the next chunk,
// loaded from HBM straight into LDS while the current chunk is processed; each
// wave loads, and later reads, only its own blocks (element j * NT + tid is
// window block j * NT + tid), so no barrier guards the stage.
template <int DT, bool HASV, bool TWO, int NT, int KPT_ = 0>
struct PartLds {
  using Cfg = PartCfg<DT, HASV, TWO, NT, KPT_>;
  static constexpr bool STAGE = TWO ? kStageTwo : kStageOne;
  uint32_t cnt[2][8][Cfg::NW];
  uint32_t sh_part;
  uint4 stage[STAGE ? Cfg::NLOAD * NT : 1];
};

// Partition of chunks [t0, t1) of the chunk space of the parts segs[0..nseg)
// (each part's chunks start at its chunk_begin; parts whose pass type is not
// TWO are skipped), workgroup of NT threads.  ctr: the parts' counter lines.
// WIDE: some part may span 4 GiB or more of keys or payloads.  SP: pointer to
// the records (constant address space when they are read-only for the kernel).
template <int DT, bool HASV, bool WIDE, bool TWO, int NT, int KPT_ = 0, bool DBG = false, typename SP>
__device__ __attribute__((always_inline)) inline void partition_chunks(
    const Ctx &c, SP segs, unsigned long long *ctr, uint32_t nseg, uint32_t t0, uint32_t t1,
    PartLds<DT, HASV, TWO, NT, KPT_> &L) {
  using Cfg = PartCfg<DT, HASV, TWO, NT, KPT_>;
  using B = typename Cfg::B;
  using C = typename Codec<DT>::C;
  // keys staged through LDS (the next chunk's loads in flight during this one)
  constexpr bool STAGE = PartLds<DT, HASV, TWO, NT, KPT_>::STAGE;
  constexpr int NW = Cfg::NW, VEC = Cfg::VEC, KPT = Cfg::KPT;
  constexpr int NLOAD = Cfg::NLOAD, KB = Cfg::KB;
  constexpr uint64_t CH = Cfg::CH;
  auto &cnt = L.cnt;
  auto &sh_part = L.sh_part;
  auto &stage = L.stage;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;

  // part containing chunk t0: 64-ary search by wave 0
  if (w == 0) {
    uint32_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
      const uint32_t step = (hi - lo + 63) / 64;
      const uint32_t probe = lo + lane * step;
      const bool ok = probe < hi && segs[probe].chunk_begin <= t0;
      const unsigned long long m = __ballot(ok);
      const uint32_t best = 63u - (uint32_t)__clzll((long long)m);
      const uint32_t nlo = lo + best * step;
      hi = (hi - nlo < step) ? hi : nlo + step;
      lo = nlo;
    }
    if (lane == 0) sh_part = lo;
  }
  __syncthreads();
  uint32_t pi = __builtin_amdgcn_readfirstlane(sh_part);

  // first chunk >= t of this kernel's pass type (t1 if none); p: its part
  auto advance = [&](uint32_t t, uint32_t &p) __attribute__((always_inline)) -> uint32_t {
    while (t < t1) {
      while (p + 1 < nseg && segs[p + 1].chunk_begin <= t) p++;
      if (((segs[p].flags & kSegTwo) != 0) == TWO) return t;
      t = p + 1 < nseg ? segs[p + 1].chunk_begin : t1;   // skip the rest of the part
    }
    return t1;
  };
  // chunk window [W, W + CH) in absolute key coordinates of the buffer holding
  // the part; the keys of the part occupy window indices [lo, hi), and win is
  // the window's first 16-byte block as an address (it may lie before the
  // buffer's start: only blocks that hold keys of the part are ever loaded)
  struct Win { const uint4 *win; uint32_t lo, hi, skip; };   // skip: keys of the part before W
  auto window = [&](uint64_t off, uint32_t len, uint32_t flags, uint32_t cb, uint32_t t)
      __attribute__((always_inline)) -> Win {
    const B *X = (const B *)((flags & kSegInS) ? c.S : c.K);
    const uint64_t xabs0 = (uint64_t)(uintptr_t)X / KB;
    const uint64_t A0 = xabs0 + off, A1 = A0 + len;
    const uint64_t W = A0 - A0 % Cfg::LINE + (uint64_t)(t - cb) * CH;
    Win r;
    r.lo = A0 > W ? (uint32_t)(A0 - W) : 0u;
    r.hi = A1 < W + CH ? (uint32_t)(A1 - W) : (uint32_t)CH;
    r.win = (const uint4 *)(X + (int64_t)(W - xabs0));
    r.skip = A0 > W ? 0u : (uint32_t)(W - A0);
    return r;
  };
  // issue the loads of chunk t (part p) into the stage
  auto prefetch = [&](uint32_t t, uint32_t p) __attribute__((always_inline)) {
    const Win g = window(segs[p].off, segs[p].len, segs[p].flags, segs[p].chunk_begin, t);
    const bool full = g.lo == 0u && g.hi == (uint32_t)CH;
#pragma unroll
    for (int j = 0; j < NLOAD; j++) {
      const uint32_t e0 = (uint32_t)(j * NT + tid) * VEC;
      if (full || (e0 + VEC > g.lo && e0 < g.hi))
        __builtin_amdgcn_global_load_lds((const void *)(g.win + j * NT + tid),
                                         (__attribute__((address_space(3))) void *)(stage + j * NT + w * kWave),
                                         16, 0, 0);
    }
  };

  // look-ahead sums (below | equal << 32) of the current part, kept by wave 0
  // (lane k: the k-th side / grandchild) until the part's last chunk here
  unsigned long long look = 0;
  uint32_t t = advance(t0, pi);
  if constexpr (STAGE) {
    if (t < t1) prefetch(t, pi);
  }
  while (t < t1) {
    const int bf = (int)((t - t0) & 1u);
    const Seg s = load_seg(segs + pi);
    uint32_t pn = pi;
    const uint32_t tn = advance(t + 1, pn);
    // source X (where the part is) and destination Y (the other buffer)
    const bool odd = (s.flags & kSegInS) != 0;
    B *Y = (B *)(odd ? c.K : c.S);
    const uint32_t *VX = odd ? c.VS : c.V;
    uint32_t *VY = odd ? c.V : c.VS;
    const Win g = window(s.off, s.len, s.flags, s.chunk_begin, t);
    const uint32_t lo = g.lo, hi = g.hi;
    // payloads from window index lo on (part index max(W - A0, 0) on)
    const uint32_t *VXp = VX + s.off + g.skip;
    const uint32_t rel0 = tid * VEC - lo;   // window index - lo, modulo 2^32
    const uint32_t wlen = hi - lo;
    B *Yp = Y + s.off;

    // keys (and payloads) of this thread: KPT items, VEC consecutive per load
    auto load = [&](auto full_tag, B (&key)[KPT], uint32_t (&val)[HASV ? KPT : 1]) __attribute__((always_inline)) {
      constexpr bool FULL = decltype(full_tag)::value;
      // per-load offsets recomputed each chunk from an opaque copy of the thread
      // index: hoisted out of the chunk loop they held a register each (the
      // two-level kernel for 4-byte keys: 96 -> 73 registers)
      uint32_t tv = tid;
      opaque_v(tv);
      const uint4 *wv0 = g.win + tv;
#pragma unroll
      for (int j = 0; j < NLOAD; j++) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if constexpr (STAGE) {
          // blocks outside the part hold stale values: the range masks drop them
          v = stage[j * NT + tid];
        } else {
          const uint32_t e0 = (uint32_t)(j * NT + tv) * VEC;
          if (FULL || (e0 + VEC > lo && e0 < hi)) v = wv0[j * NT];
        }
        if constexpr (KB == 4) {
          key[j * VEC + 0] = v.x; key[j * VEC + 1] = v.y; key[j * VEC + 2] = v.z; key[j * VEC + 3] = v.w;
        } else {
          key[j * VEC + 0] = (uint64_t)v.x | ((uint64_t)v.y << 32);
          key[j * VEC + 1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
        }
        if constexpr (HASV) {
#pragma unroll
          for (int q = 0; q < VEC; q++) {
            const uint32_t r = rel0 + (uint32_t)(j * NT * VEC + q);
            // unconditional (index clamped into the part): loads stay in flight together
            val[j * VEC + q] = *at<false>(VXp, (FULL || r < wlen) ? r : 0u);
          }
        }
      }
      if constexpr (STAGE) {
        // the stage is free once its blocks are in registers: load the next chunk
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        if (tn < t1) prefetch(tn, pn);
      }
    };
    // item it of every thread lies past the part's end (partial chunks; the
    // same for the whole workgroup): skipped by a uniform branch, which saves a
    // part smaller than a chunk most of the chunk's work
    auto past_part = [&](auto full_tag, int it) __attribute__((always_inline)) -> bool {
      constexpr bool FULL = decltype(full_tag)::value;
      if constexpr (FULL) return false;
      else return (uint32_t)((it / VEC) * NT * VEC) >= hi;
    };
    // range mask of item it (partial chunks): the lanes whose key is in the part
    auto range_mask = [&](auto full_tag, int it, uint32_t relc) __attribute__((always_inline)) -> unsigned long long {
      constexpr bool FULL = decltype(full_tag)::value;
      if constexpr (FULL) return ~0ull;
      else return wave_ballot(relc + (uint32_t)((it / VEC) * NT * VEC + (it % VEC)) < wlen);
    };

    // ---- one-level pass: split by piv[0] with a left and a right cursor ----
    auto body1 = [&](auto full_tag) __attribute__((always_inline)) {
      constexpr bool FULL = decltype(full_tag)::value;
      B key[KPT];
      uint32_t val[HASV ? KPT : 1];
      load(full_tag, key, val);
      C pvc = Codec<DT>::cpiv(s.piv[0]), pl = Codec<DT>::cpiv(s.piv[1]), pg = Codec<DT>::cpiv(s.piv[2]);
      uint32_t relc = rel0;
      // pass 1: this wave's class totals, and the look-ahead counts of each side
      // against its own pivot (scalar)
      uint32_t sL = 0, sG = 0, sO = 0, aLl = 0, aLe = 0, aGl = 0, aGe = 0;
      static_for<0, KPT>([&](auto I) __attribute__((always_inline)) {
        constexpr int it = decltype(I)::value;
        if (past_part(full_tag, it)) return;
        const C u = Codec<DT>::ckey(key[it]);
        const unsigned long long om = range_mask(full_tag, it, relc);
        const unsigned long long lm = wave_ballot(u < pvc) & om, gm = wave_ballot(u > pvc) & om;
        sL += (uint32_t)__popcll(lm);
        sG += (uint32_t)__popcll(gm);
        if constexpr (HASV && !FULL) sO += (uint32_t)__popcll(om);
        // one item at a time: deferring the sums would keep every mask live
        opaque_s(sL);
        opaque_s(sG);
        if constexpr (HASV && !FULL) opaque_s(sO);
        const C pc = pick<C>(u < pvc, pl, pg);
        const unsigned long long m1 = wave_ballot(u < pc), e1 = wave_ballot(u == pc);
        aLl += (uint32_t)__popcll(lm & m1);
        aLe += (uint32_t)__popcll(lm & e1);
        aGl += (uint32_t)__popcll(gm & m1);
        aGe += (uint32_t)__popcll(gm & e1);
        opaque_s(aLl); opaque_s(aLe); opaque_s(aGl); opaque_s(aGe);
      });
      if constexpr (HASV && FULL) sO = (uint32_t)(kWave * KPT);
      if (lane == 0) {
        cnt[bf][0][w] = sL;
        cnt[bf][1][w] = sG;
        cnt[bf][2][w] = aLl; cnt[bf][3][w] = aLe; cnt[bf][4][w] = aGl; cnt[bf][5][w] = aGe;
        if constexpr (HASV) cnt[bf][6][w] = sO - sL - sG;
      }
      __syncthreads();
      // exclusive prefix over the waves of each class; one reservation per chunk
      if (w == 0) {
        const uint32_t a = lane < (uint32_t)NW ? cnt[bf][0][lane] : 0u;
        const uint32_t b = lane < (uint32_t)NW ? cnt[bf][1][lane] : 0u;
        uint32_t e = 0;
        if constexpr (HASV) e = lane < (uint32_t)NW ? cnt[bf][6][lane] : 0u;
        const uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
        uint32_t ie = 0;
        if constexpr (HASV) ie = wave_incl_scan(e);
        unsigned long long *cp = ctr + (size_t)pi * kCtrStride;
        unsigned long long rb = 0;
        uint32_t re = 0;
        if (lane == (uint32_t)NW - 1) {
          rb = atomicAdd(cp + kCtrA, ((unsigned long long)ib << 32) | ia);
          if constexpr (HASV) re = (uint32_t)atomicAdd(cp + kCtrE, (unsigned long long)ie);
        }
        // look-ahead totals: lane 0 the < side, lane 1 the > side
        if (lane < 2) {
          uint32_t tl = 0, te = 0;
          for (int q = 0; q < NW; q++) { tl += cnt[bf][2 + 2 * lane][q]; te += cnt[bf][3 + 2 * lane][q]; }
          look += ((unsigned long long)te << 32) | tl;
        }
        // < keys fill from the left cursor, > keys from the right cursor
        // (the reserved block ends where the previous reservations began)
        rb = __shfl(rb, NW - 1);
        const uint32_t totG = __shfl(ib, NW - 1);
        if constexpr (HASV) re = __shfl(re, NW - 1);
        if (lane < (uint32_t)NW) {
          cnt[bf][0][lane] = (uint32_t)rb + ia - a;
          cnt[bf][1][lane] = s.len - (uint32_t)(rb >> 32) - totG + ib - b;
          if constexpr (HASV) cnt[bf][6][lane] = re + ie - e;
        }
      }
      __syncthreads();
      uint32_t runL = __builtin_amdgcn_readfirstlane(cnt[bf][0][w]);
      uint32_t runG = __builtin_amdgcn_readfirstlane(cnt[bf][1][w]);
      uint32_t runE = 0;
      if constexpr (HASV) runE = __builtin_amdgcn_readfirstlane(cnt[bf][6][w]);
      uint32_t *VYp = VY + s.off;
      uint32_t *VEp = c.VE + s.off;
      // codes are recomputed from the keys (no second register copy)
      static_for<0, KPT>([&](auto I) __attribute__((always_inline)) { opaque_v(key[decltype(I)::value]); });
      // pass 2: the comparisons are recomputed rather than kept (2 x KPT wave
      // masks do not fit in scalar registers); the opaque copies stop the
      // compiler from keeping them
      opaque_v(pvc);
      opaque_v(relc);
      static_for<0, KPT>([&](auto I) __attribute__((always_inline)) {
        constexpr int it = decltype(I)::value;
        if (past_part(full_tag, it)) return;
        const C u = Codec<DT>::ckey(key[it]);
        const unsigned long long om = range_mask(full_tag, it, relc);
        bool lt = u < pvc, gt = u > pvc;
        if constexpr (!FULL) {
          const bool ok = relc + (uint32_t)((it / VEC) * NT * VEC + (it % VEC)) < wlen;
          lt = lt && ok;
          gt = gt && ok;
        }
        const unsigned long long lm = wave_ballot(lt), gm = wave_ballot(gt);
        uint32_t posL = runL + mbcnt(lm), posG = runG + mbcnt(gm);
        opaque_v(posL);   // select the position, not the masks
        opaque_v(posG);
        const uint32_t pos = pick<uint32_t>(lt, posL, posG);
        runL += (uint32_t)__popcll(lm);
        runG += (uint32_t)__popcll(gm);
        if (lt || gt) {
          *at<WIDE>(Yp, pos) = key[it];
          if constexpr (HASV) *at<WIDE>(VYp, pos) = val[it];
          if constexpr (DBG) dbg_store(c, odd, s.off + pos, s.depth);
        }
        if constexpr (HASV) {
          const unsigned long long em = om & ~(lm | gm);
          if ((em >> lane) & 1ull) *at<WIDE>(VEp, runE + mbcnt(em)) = val[it];
          runE += (uint32_t)__popcll(em);
        }
        __builtin_amdgcn_sched_barrier(0);
      });
    };

    // ---- two-level pass: regions of piv[0] placed exactly, each split by its
    // own pivot with two cursors; payloads move with their keys, and those of
    // the keys equal to piv[0], piv[1], piv[2] are staged in VE at [nlt, ...),
    // [0, ...) and [nlt + neq, ...) of the part (disjoint: the band of piv[1]
    // lies inside the < region) for the band fills ----
    auto body2 = [&](auto full_tag) __attribute__((always_inline)) {
      B key[KPT];
      uint32_t val[HASV ? KPT : 1];
      load(full_tag, key, val);
      C p0 = Codec<DT>::cpiv(s.piv[0]), pl = Codec<DT>::cpiv(s.piv[1]), pg = Codec<DT>::cpiv(s.piv[2]);
      C pll = Codec<DT>::cpiv(s.piv[3]), plg = Codec<DT>::cpiv(s.piv[4]);
      C pgl = Codec<DT>::cpiv(s.piv[5]), pgg = Codec<DT>::cpiv(s.piv[6]);
      uint32_t relc = rel0;
      // pass 1: the four grandchild classes (<<, <>, ><, >>) and, with payloads,
      // the three equal classes (= piv[0], = piv[1], = piv[2]) (scalar)
      uint32_t n0 = 0, n1 = 0, n2 = 0, n3 = 0, z0 = 0, z1 = 0, z2 = 0;
      static_for<0, KPT>([&](auto I) __attribute__((always_inline)) {
        constexpr int it = decltype(I)::value;
        if (past_part(full_tag, it)) return;
        const C u = Codec<DT>::ckey(key[it]);
        const unsigned long long om = range_mask(full_tag, it, relc);
        const bool lt0 = u < p0;
        const unsigned long long ma = wave_ballot(lt0) & om, mb = wave_ballot(u > p0) & om;
        const C pc = pick<C>(lt0, pl, pg);
        const unsigned long long m1l = wave_ballot(u < pc), m1g = wave_ballot(u > pc);
        n0 += (uint32_t)__popcll(ma & m1l); n1 += (uint32_t)__popcll(ma & m1g);
        n2 += (uint32_t)__popcll(mb & m1l); n3 += (uint32_t)__popcll(mb & m1g);
        opaque_s(n0); opaque_s(n1); opaque_s(n2); opaque_s(n3);
        if constexpr (HASV) {
          const unsigned long long mn = ~(m1l | m1g);
          z0 += (uint32_t)__popcll(om & ~(ma | mb));
          z1 += (uint32_t)__popcll(ma & mn);
          z2 += (uint32_t)__popcll(mb & mn);
          opaque_s(z0); opaque_s(z1); opaque_s(z2);
        }
      });
      if (lane == 0) {
        cnt[bf][0][w] = n0; cnt[bf][1][w] = n1; cnt[bf][2][w] = n2; cnt[bf][3][w] = n3;
        if constexpr (HASV) { cnt[bf][4][w] = z0; cnt[bf][5][w] = z1; cnt[bf][6][w] = z2; }
      }
      __syncthreads();
      if (w == 0) {
        constexpr int K = HASV ? 7 : 4;
        uint32_t x[K], ix[K], tt[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
          x[k] = lane < (uint32_t)NW ? cnt[bf][k][lane] : 0u;
          ix[k] = wave_incl_scan(x[k]);
          tt[k] = __shfl(ix[k], NW - 1);
        }
        unsigned long long *cp = ctr + (size_t)pi * kCtrStride;
        unsigned long long ra = 0, rb = 0, re0 = 0, re12 = 0;
        if (lane == (uint32_t)NW - 1) {
          ra = atomicAdd(cp + kCtrA, ((unsigned long long)ix[1] << 32) | ix[0]);
          rb = atomicAdd(cp + kCtrB, ((unsigned long long)ix[3] << 32) | ix[2]);
          if constexpr (HASV) {
            re0 = atomicAdd(cp + kCtrE, (unsigned long long)ix[4]);
            re12 = atomicAdd(cp + kCtrE12, ((unsigned long long)ix[6] << 32) | ix[5]);
          }
        }
        ra = __shfl(ra, NW - 1);
        rb = __shfl(rb, NW - 1);
        if constexpr (HASV) {
          re0 = __shfl(re0, NW - 1);
          re12 = __shfl(re12, NW - 1);
        }
        const uint32_t g0 = s.nlt + s.neq;
        // the regions come from the previous pass's counts: a chunk that would
        // overfill one reports an internal error (its stores are also bounded)
        bool bad = (uint64_t)(uint32_t)ra + tt[0] + (uint32_t)(ra >> 32) + tt[1] > s.nlt ||
                   (uint64_t)(uint32_t)rb + tt[2] + (uint32_t)(rb >> 32) + tt[3] + g0 > s.len;
        if constexpr (HASV)
          bad = bad || (uint64_t)(uint32_t)re0 + tt[4] > s.neq ||
                (uint64_t)(uint32_t)re12 + tt[5] > s.nlt ||
                (uint64_t)(uint32_t)(re12 >> 32) + tt[6] + g0 > s.len;
        if (lane == 0 && bad) atomicOr(c.err, kErrCount);
        if (lane < (uint32_t)NW) {
          // << from the start of the < region, <> as blocks from its end, ><
          // from the start of the > region, >> as blocks from the part's end
          cnt[bf][0][lane] = (uint32_t)ra + ix[0] - x[0];
          cnt[bf][1][lane] = s.nlt - (uint32_t)(ra >> 32) - tt[1] + ix[1] - x[1];
          cnt[bf][2][lane] = g0 + (uint32_t)rb + ix[2] - x[2];
          cnt[bf][3][lane] = s.len - (uint32_t)(rb >> 32) - tt[3] + ix[3] - x[3];
          if constexpr (HASV) {
            // staging offsets (from the part's start) of the equal classes
            cnt[bf][4][lane] = s.nlt + (uint32_t)re0 + ix[4] - x[4];
            cnt[bf][5][lane] = (uint32_t)re12 + ix[5] - x[5];
            cnt[bf][6][lane] = g0 + (uint32_t)(re12 >> 32) + ix[6] - x[6];
          }
        }
      }
      __syncthreads();
      uint32_t r0 = __builtin_amdgcn_readfirstlane(cnt[bf][0][w]);
      uint32_t r1 = __builtin_amdgcn_readfirstlane(cnt[bf][1][w]);
      uint32_t r2 = __builtin_amdgcn_readfirstlane(cnt[bf][2][w]);
      uint32_t r3 = __builtin_amdgcn_readfirstlane(cnt[bf][3][w]);
      uint32_t y0 = 0, y1 = 0, y2 = 0;
      if constexpr (HASV) {
        y0 = __builtin_amdgcn_readfirstlane(cnt[bf][4][w]);
        y1 = __builtin_amdgcn_readfirstlane(cnt[bf][5][w]);
        y2 = __builtin_amdgcn_readfirstlane(cnt[bf][6][w]);
      }
      uint32_t *VYp = VY + s.off;
      uint32_t *VEp = c.VE + s.off;
      // codes are recomputed from the keys (no second register copy)
      static_for<0, KPT>([&](auto I) __attribute__((always_inline)) { opaque_v(key[decltype(I)::value]); });
      // pass 2: stores, and the look-ahead counts of the grandchildren against
      // piv[3..6]: per lane, 8-bit counters packed by grandchild (byte k: keys
      // of grandchild k below / equal to its pivot; at most KPT <= 255 per lane),
      // reduced over the wave and the workgroup after the pass
      static_assert(KPT <= 255, "packed look-ahead counters");
      uint32_t accL = 0, accE = 0;
      // pivots selected per lane live in vector registers (a select takes at
      // most one scalar operand)
      opaque_v(pl); opaque_v(pg);
      opaque_v(pll); opaque_v(plg); opaque_v(pgl); opaque_v(pgg);
      opaque_v(p0);
      opaque_v(relc);
      static_for<0, KPT>([&](auto I) __attribute__((always_inline)) {
        constexpr int it = decltype(I)::value;
        if (past_part(full_tag, it)) return;
        const C u = Codec<DT>::ckey(key[it]);
        const unsigned long long om = range_mask(full_tag, it, relc);
        const bool lt0 = u < p0, gt0 = u > p0;
        const C pc = pick<C>(lt0, pl, pg);
        const bool lt1 = u < pc, gt1 = u > pc;
        const unsigned long long ma = wave_ballot(lt0) & om, mb = wave_ballot(gt0) & om;
        const unsigned long long m1l = wave_ballot(lt1), m1g = wave_ballot(gt1);
        const unsigned long long q0 = ma & m1l, q1 = ma & m1g, q2 = mb & m1l, q3 = mb & m1g;
        uint32_t x0 = r0 + mbcnt(q0), x1 = r1 + mbcnt(q1), x2 = r2 + mbcnt(q2), x3 = r3 + mbcnt(q3);
        opaque_v(x0); opaque_v(x1); opaque_v(x2); opaque_v(x3);
        const uint32_t pos = pick<uint32_t>(lt0, pick<uint32_t>(lt1, x0, x1), pick<uint32_t>(lt1, x2, x3));
        r0 += (uint32_t)__popcll(q0); r1 += (uint32_t)__popcll(q1);
        r2 += (uint32_t)__popcll(q2); r3 += (uint32_t)__popcll(q3);
        const bool in = ((om >> lane) & 1ull) && (lt0 || gt0) && (lt1 || gt1);
        const C pq = pick<C>(lt0, pick<C>(lt1, pll, plg), pick<C>(lt1, pgl, pgg));
        const uint32_t one = 1u << (pick<uint32_t>(gt0, 16u, 0u) + pick<uint32_t>(gt1, 8u, 0u));
        accL += (in && u < pq) ? one : 0u;
        accE += (in && u == pq) ? one : 0u;
        // counted before the store: the masks of this item end here
        opaque_v(accL); opaque_v(accE);
        if constexpr (HASV) {
          // equal classes: payloads staged for the band fills
          const unsigned long long mn = ~(m1l | m1g);
          const unsigned long long e0 = om & ~(ma | mb), e1 = ma & mn, e2 = mb & mn;
          uint32_t w0 = y0 + mbcnt(e0), w1 = y1 + mbcnt(e1), w2 = y2 + mbcnt(e2);
          opaque_v(w0); opaque_v(w1); opaque_v(w2);
          const uint32_t epos = pick<uint32_t>(lt0, w1, pick<uint32_t>(gt0, w2, w0));
          y0 += (uint32_t)__popcll(e0); y1 += (uint32_t)__popcll(e1); y2 += (uint32_t)__popcll(e2);
          if ((((e0 | e1 | e2) >> lane) & 1ull) && epos < s.len) *at<WIDE>(VEp, epos) = val[it];
          opaque_s(y0); opaque_s(y1); opaque_s(y2);
        }
        if (in && pos < s.len) {
          *at<WIDE>(Yp, pos) = key[it];
          if constexpr (HASV) *at<WIDE>(VYp, pos) = val[it];
          if constexpr (DBG) dbg_store(c, odd, s.off + pos, s.depth);
        }
        opaque_s(r0); opaque_s(r1); opaque_s(r2); opaque_s(r3);
        // four items at a time (keys only; with payloads one): enough overlap to
        // hide the compare-to-mask latency, few enough masks live to stay in
        // scalar registers
        if constexpr (HASV || it % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      });
      // widen to 16-bit fields (grandchildren 0 and 2 | 1 and 3; a chunk has at
      // most 2^16 - 1 keys) and sum over the wave
      static_assert(CH < 65536, "16-bit look-ahead sums");
      uint32_t f[4] = {accL & 0x00FF00FFu, (accL >> 8) & 0x00FF00FFu,
                       accE & 0x00FF00FFu, (accE >> 8) & 0x00FF00FFu};
#pragma unroll
      for (int k = 0; k < 4; k++) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) f[k] += shfl_xor_u32(f[k], o);
      }
      if (lane == 0) {
        cnt[bf][4][w] = f[0]; cnt[bf][5][w] = f[1]; cnt[bf][6][w] = f[2]; cnt[bf][7][w] = f[3];
      }
      __syncthreads();
      if (w == 0 && lane < 4) {
        // grandchild q = lane: field (q & 2) * 8 of word q & 1
        uint32_t tl = 0, te = 0;
        for (int q = 0; q < NW; q++) { tl += cnt[bf][4 + (lane & 1)][q]; te += cnt[bf][6 + (lane & 1)][q]; }
        const int sh = (lane & 2) ? 16 : 0;
        tl = (tl >> sh) & 0xFFFFu;
        te = (te >> sh) & 0xFFFFu;
        look += ((unsigned long long)te << 32) | tl;
      }
    };

    const bool full = lo == 0u && hi == (uint32_t)CH;
    if constexpr (TWO) {
      if (full) body2(std::true_type{});
      else body2(std::false_type{});
    } else {
      if (full) body1(std::true_type{});
      else body1(std::false_type{});
    }
    // the look-ahead sums of a run of chunks of one part go out together
    if (w == 0 && (tn >= t1 || pn != pi)) {
      if (lane < (TWO ? 4u : 2u) && look) atomicAdd(ctr + (size_t)pi * kCtrStride + kCtrLook + lane, look);
      look = 0;
    }
    t = tn;
    pi = pn;
  }
}

// The two-level instance for 4-byte keys without payload asks for 7 waves per
// SIMD (at most 72 registers, no spills): its chunks are latency-bound, and 2^28
// int32 passes take 4.9 ms at 7 workgroups per CU, 5.0 at 6 and 5.05 at 5.
template <int DT, bool HASV, bool TWO, int WGX, bool DBG>
constexpr int part_waves() {
  return (TWO && !HASV && sizeof(typename Codec<DT>::B) == 4 && WGX == 1 && !DBG) ? 7 : 1;
}

// One partition level: every chunk of every part of level d whose pass type is
// TWO (two-level parts); the parts of the other type are skipped (a kernel per
// type, so each has the registers, and the occupancy, its own work needs).
// WGX = 2: twice the threads per workgroup, half the keys per thread (the same
// chunks: the planning's chunk counts hold for either).
template <int DT, bool HASV, bool WIDE, bool TWO, int WGX = 1, bool DBG = false>
__global__ __launch_bounds__((TWO ? kPartNT2 : kPartNT1) * WGX)
__attribute__((amdgpu_waves_per_eu(part_waves<DT, HASV, TWO, WGX, DBG>()))) void k_partition(Ctx c, int d) {
  constexpr int NT = (TWO ? kPartNT2 : kPartNT1) * WGX;
  constexpr int KPT_ = WGX == 1 ? 0 : PartCfg<DT, HASV, TWO>::KPT / WGX;
  static_assert(PartCfg<DT, HASV, TWO, NT, KPT_>::CH == PartCfg<DT, HASV, TWO>::CH, "chunk");
  __shared__ PartLds<DT, HASV, TWO, NT, KPT_> L;
  const unsigned long long packed = c.lvl[d].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  const uint32_t nch = (uint32_t)(packed & kTileMask);
  // a failed capacity check leaves the count above the records written: stop
  if (nch == 0 || nseg == 0 || nseg > c.seg_cap) return;
  const uint32_t per = (nch + gridDim.x - 1) / gridDim.x;
  const uint32_t t0 = blockIdx.x * per;
  if (t0 >= nch) return;
  const uint32_t t1 = (nch - t0 < per) ? nch : t0 + per;
  // the records of level d are read-only here (written by the previous level's
  // planning): read through the constant address space, so that uniform reads
  // become scalar loads even after this kernel's own stores
  const CSeg *segs = (const CSeg *)((d & 1) ? c.seg1 : c.seg0);
  unsigned long long *ctr = (d & 1) ? c.ctr1 : c.ctr0;
  partition_chunks<DT, HASV, WIDE, TWO, NT, KPT_, DBG>(c, segs, ctr, nseg, t0, t1, L);
}

// After level d: bands, small children, next-level parts with pivots (a wave per
// part, workgroup-uniform iterations so the workgroup can reserve together).
// A one-level part leaves its < child (slot 4i), its > child (slot 4i+3) and the
// band of piv[0] (band slot 3i+1); a two-level part leaves four grandchildren
// (slots 4i..4i+3) and three bands: piv[1] inside the < region (3i), piv[0]
// (3i+1), piv[2] inside the > region (3i+2).  Unused slots are written empty.
template <int DT, bool HASV>
__global__ __launch_bounds__(kPlanNT) void k_plan(Ctx c, int d) {
  __shared__ uint32_t hist[kPlanNW][256];
  __shared__ PendLds pend;
  const unsigned long long packed = c.lvl[d].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  if (nseg > c.seg_cap) return;
  const Seg *segs = (d & 1) ? c.seg1 : c.seg0;
  const unsigned long long *ctr = (d & 1) ? c.ctr1 : c.ctr0;
  const uint32_t wv = threadIdx.x / kWave, lane = threadIdx.x & 63u;
  if (lane == 0) { pend.n[wv] = 0; pend.ch[wv] = 0; pend.keys[wv] = 0; }
  __syncthreads();
  unsigned long long small_parts = 0, small_keys = 0, band_keys = 0;
  const int next = level_after(c, d);
  for (uint32_t base = blockIdx.x * kPlanNW; base < nseg; base += gridDim.x * kPlanNW) {
    const uint32_t si = base + wv;
    if (si < nseg) {
      const Seg s = segs[si];
      const unsigned long long *cp = ctr + (size_t)si * kCtrStride;
      const bool out_s = (s.flags & kSegInS) == 0;     // children live in the other buffer
      if (s.flags & kSegTwo) {
        const unsigned long long ca = cp[kCtrA], cb = cp[kCtrB];
        const uint32_t nll = (uint32_t)ca, nlg = (uint32_t)(ca >> 32);
        const uint32_t ngl = (uint32_t)cb, ngg = (uint32_t)(cb >> 32);
        const uint32_t nlt = s.nlt, neq = s.neq, g0 = nlt + neq;
        const uint32_t ele = nlt - nll - nlg, egt = (s.len - g0) - ngl - ngg;
        if ((uint64_t)nll + nlg > nlt || (uint64_t)g0 + ngl + ngg > s.len) {
          // counts that do not fit the regions (a bug): report, emit nothing
          if (lane == 0) {
            atomicOr(c.err, kErrCount);
            FinItem z;
            z.off = 0; z.src = 0; z.pivot = 0; z.len = 0; z.kind = 0;
            for (int k = 0; k < 3; k++) c.band[3 * si + k] = z;
            for (int k = 0; k < 4; k++) put_small(c, 4 * si + k, 0, 0, false, s.req);
          }
        } else {
        if (lane == 0) {
          // payloads of each band were staged at [0, ...), [nlt, ...), [g0, ...)
          put_band(c, d, 3 * si + 0, s.off + nll, s.off, ele, s.piv[1], s.req);
          put_band(c, d, 3 * si + 1, s.off + nlt, s.off + nlt, neq, s.piv[0], s.req);
          put_band(c, d, 3 * si + 2, s.off + g0 + ngl, s.off + g0, egt, s.piv[2], s.req);
          band_keys += (unsigned long long)ele + neq + egt;
        }
        const uint64_t coff[4] = {s.off, s.off + nlt - nlg, s.off + g0, s.off + s.len - ngg};
        const uint32_t clen[4] = {nll, nlg, ngl, ngg};
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const unsigned long long la = cp[kCtrLook + k];
          child<DT, HASV>(c, 4 * si + k, coff[k], clen[k], child_depth(s.depth, 2, s.len, clen[k], s.dmax),
                          s.dmax, s.req, out_s, true,
                          s.piv[3 + k], (uint32_t)la, (uint32_t)(la >> 32), hist[wv], pend, wv,
                          small_parts, small_keys);
        }
        }
      } else {
        const unsigned long long cv = cp[kCtrA];
        const uint32_t L = (uint32_t)cv, G = (uint32_t)(cv >> 32);
        const uint32_t E = s.len - L - G;
        if (lane == 0) {
          FinItem z;
          z.off = 0; z.src = 0; z.pivot = 0; z.len = 0; z.kind = 0;
          c.band[3 * si + 0] = z;
          c.band[3 * si + 2] = z;
          put_band(c, d, 3 * si + 1, s.off + L, s.off, E, s.piv[0], s.req);
          band_keys += E;
          put_small(c, 4 * si + 1, 0, 0, false, s.req);
          put_small(c, 4 * si + 2, 0, 0, false, s.req);
        }
        const unsigned long long la = cp[kCtrLook + 0], ga = cp[kCtrLook + 1];
        child<DT, HASV>(c, 4 * si, s.off, L, child_depth(s.depth, 1, s.len, L, s.dmax), s.dmax, s.req,
                        out_s, true, s.piv[1],
                        (uint32_t)la, (uint32_t)(la >> 32), hist[wv], pend, wv, small_parts,
                        small_keys);
        child<DT, HASV>(c, 4 * si + 3, s.off + s.len - G, G, child_depth(s.depth, 1, s.len, G, s.dmax),
                        s.dmax, s.req, out_s, true,
                        s.piv[2], (uint32_t)ga, (uint32_t)(ga >> 32), hist[wv], pend, wv,
                        small_parts, small_keys);
      }
    }
    flush_parts<DT, HASV>(c, next, pend);
  }
  if (lane == 0) {
    stat_add(c, kStSmallParts, small_parts);
    stat_add(c, kStSmallKeys, small_keys);
    stat_add(c, kStBandKeys, band_keys);
  }
}

// ---- small-part sort: bitonic network in registers ------------------------------

// Records of the small-part sort: the code, plus (with payloads) the local
// index, so that padding sorts after every real key and payloads can follow.
template <typename B, bool HASV> struct Rec;
template <typename B> struct Rec<B, false> {
  using T = B;
  __device__ static inline T make(B code, uint32_t) { return code; }
  __device__ static inline T pad() { return ~(B)0; }
  __device__ static inline B code(T r) { return r; }
  __device__ static inline uint32_t idx(T) { return 0; }
  __device__ static inline bool less(T a, T b) { return a < b; }
  __device__ static inline T sel(bool c, T a, T b) { return c ? a : b; }
};
template <> struct Rec<uint32_t, true> {
  using T = uint64_t;
  __device__ static inline T make(uint32_t code, uint32_t i) { return ((uint64_t)code << 32) | i; }
  __device__ static inline T pad() { return ~0ull; }
  __device__ static inline uint32_t code(T r) { return (uint32_t)(r >> 32); }
  __device__ static inline uint32_t idx(T r) { return (uint32_t)r; }
  __device__ static inline bool less(T a, T b) { return a < b; }
  __device__ static inline T sel(bool c, T a, T b) { return c ? a : b; }
};
struct R64 { uint64_t k; uint32_t i; uint32_t pad; };
template <> struct Rec<uint64_t, true> {
  using T = R64;
  __device__ static inline T make(uint64_t code, uint32_t i) { T r; r.k = code; r.i = i; r.pad = 0; return r; }
  __device__ static inline T pad() { T r; r.k = ~0ull; r.i = ~0u; r.pad = 0; return r; }
  __device__ static inline uint64_t code(T r) { return r.k; }
  __device__ static inline uint32_t idx(T r) { return r.i; }
  __device__ static inline bool less(T a, T b) { return a.k < b.k || (a.k == b.k && a.i < b.i); }
  // field by field: a select of the whole struct can be lowered through memory
  __device__ static inline T sel(bool c, T a, T b) {
    T r;
    r.k = c ? a.k : b.k;
    r.i = c ? a.i : b.i;
    r.pad = 0;
    return r;
  }
};

// Partner exchange inside a wave: the value of lane (lane ^ DD).  Distances
// 1, 2, 4 and 8 use DPP moves (quad_perm, row_mirror, row_half_mirror), 16 and
// 32 the gfx950 row swaps (v_permlane16_swap / v_permlane32_swap: each returns
// the lower and the upper lane's value of the pair): VALU only, no LDS
// traffic.  DD = 0: ds_bpermute with the byte address `addr`.
template <int CTRL>
__device__ inline uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
template <int DD>
__device__ inline uint32_t xch(uint32_t v, int addr) {
  if constexpr (DD == 1) return dpp32<0xB1>(v);                 // quad_perm(1,0,3,2)
  else if constexpr (DD == 2) return dpp32<0x4E>(v);            // quad_perm(2,3,0,1)
  else if constexpr (DD == 4) return dpp32<0x1B>(dpp32<0x141>(v));  // half_mirror, quad_perm(3,2,1,0)
  else if constexpr (DD == 8) return dpp32<0x141>(dpp32<0x140>(v)); // mirror, half_mirror
  else if constexpr (DD == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (__lane_id() & 16u) ? r[0] : r[1];
  } else if constexpr (DD == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (__lane_id() & 32u) ? r[0] : r[1];
  } else return (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)v);
}
// The values of the lower and the upper lane of this lane's pair (lane and
// lane ^ DD, DD = 16 or 32), from one row swap per 32-bit word.
template <int DD>
__device__ inline void swap_pair(uint32_t v, uint32_t &lo, uint32_t &hi) {
  if constexpr (DD == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    lo = r[0]; hi = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    lo = r[0]; hi = r[1];
  }
}
template <int DD>
__device__ inline void swap_pair(uint64_t v, uint64_t &lo, uint64_t &hi) {
  uint32_t l0, h0, l1, h1;
  swap_pair<DD>((uint32_t)v, l0, h0);
  swap_pair<DD>((uint32_t)(v >> 32), l1, h1);
  lo = ((uint64_t)l1 << 32) | l0;
  hi = ((uint64_t)h1 << 32) | h0;
}

template <int DD>
__device__ inline uint64_t xch(uint64_t v, int addr) {
  const uint32_t lo = xch<DD>((uint32_t)v, addr), hi = xch<DD>((uint32_t)(v >> 32), addr);
  return ((uint64_t)hi << 32) | lo;
}
template <int DD>
__device__ inline R64 xch(R64 v, int addr) {
  R64 r;
  r.k = xch<DD>(v.k, addr);
  r.i = xch<DD>(v.i, addr);
  r.pad = 0;
  return r;
}
template <int DD>
__device__ inline void swap_pair(R64 v, R64 &lo, R64 &hi) {
  swap_pair<DD>(v.k, lo.k, hi.k);
  swap_pair<DD>(v.i, lo.i, hi.i);
  lo.pad = 0; hi.pad = 0;
}

// keys per lane of the small-part sort, bounded by registers: 32 for 4-byte
// records, 16 for 8-byte, 8 for 16-byte
template <typename T> constexpr int max_e() { return sizeof(T) <= 4 ? 32 : (sizeof(T) <= 8 ? 16 : 8); }

template <typename R>
__device__ inline void cas_asc(typename R::T &a, typename R::T &b) {
  const bool sw = R::less(b, a);
  const typename R::T lo = R::sel(sw, b, a), hi = R::sel(sw, a, b);
  a = lo; b = hi;
}

// full ascending bitonic sort of the E registers of one thread
template <typename R, int E>
__device__ inline void sort_regs_asc(typename R::T (&v)[E]) {
#pragma unroll
  for (int k = 2; k <= E; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < E; i++) {
        const int p = i ^ j;
        if (p > i) {
          if ((i & k) == 0) cas_asc<R>(v[i], v[p]);
          else cas_asc<R>(v[p], v[i]);
        }
      }
    }
  }
}

// ascending merge of a bitonic sequence held in the E registers
template <typename R, int E>
__device__ inline void merge_regs_asc(typename R::T (&v)[E]) {
#pragma unroll
  for (int j = E >> 1; j > 0; j >>= 1) {
#pragma unroll
    for (int i = 0; i < E; i++)
      if ((i & j) == 0) cas_asc<R>(v[i], v[i + j]);
  }
}

// median of three 32-bit values (one v_med3_u32)
__device__ inline uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));
}

// merge of a bitonic sequence held in the E registers, ascending or
// descending (32-bit codes: each compare-exchange as two medians with the
// direction's constants, so no reversal afterwards)
template <typename R, int E>
__device__ inline void merge_regs_dir(typename R::T (&v)[E], bool asc);

template <typename R, int E>
__device__ inline void reverse_if(typename R::T (&v)[E], bool cond) {
#pragma unroll
  for (int i = 0; i < E / 2; i++) {
    const typename R::T a = v[i], b = v[E - 1 - i];
    v[i] = R::sel(cond, b, a);
    v[E - 1 - i] = R::sel(cond, a, b);
  }
}

template <typename R, int E>
__device__ inline void merge_regs_dir(typename R::T (&v)[E], bool asc) {
  using T = typename R::T;
  if constexpr (std::is_same<T, uint32_t>::value) {
    const uint32_t c0 = asc ? 0u : ~0u, c1 = ~c0;
#pragma unroll
    for (int j = E >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < E; i++)
        if ((i & j) == 0) {
          const uint32_t a = v[i], b = v[i + j];
          v[i] = med3_u32(a, b, c0);
          v[i + j] = med3_u32(a, b, c1);
        }
    }
  } else {
    merge_regs_asc<R, E>(v);
    reverse_if<R, E>(v, !asc);
  }
}

__device__ inline uint32_t lds_pad(uint32_t x) { return x + (x >> 5); }
// lds_pad(i * NT + t) for t < NT, NT a multiple of 32: a base per thread plus a
// constant per i, which the LDS instructions take as their immediate offset (the
// compiler, not knowing t < NT, kept one register per i across parts)
template <int NT>
__device__ inline uint32_t lds_stripe(uint32_t i, uint32_t t) {
  static_assert(NT % 32 == 0, "stripe");
  return i * (uint32_t)(NT + NT / 32) + t + (t >> 5);
}

template <int NT>
__device__ inline void group_sync() {
  if constexpr (NT == kWave) wave_lds_sync();
  else __syncthreads();
}

// One compare-exchange stage against the partner lane (lane ^ DD; DD = 0 means
// "use the permute address"), permutes issued eight at a time.
template <typename R, int E, int DD>
__device__ inline void cross_stage(typename R::T (&v)[E], bool take_min, int addr) {
  using T = typename R::T;
  constexpr int GB = E < 8 ? E : 8;
  if constexpr (std::is_same<T, uint32_t>::value) {
    // 32-bit codes: the median of (mine, partner's, 0) is the smaller of the
    // two, of (mine, partner's, ~0) the larger: one instruction per record
    const uint32_t cm = take_min ? 0u : ~0u;
#pragma unroll
    for (int i = 0; i < E; i++) {
      if constexpr (DD == 16 || DD == 32) {
        uint32_t lo, hi;
        swap_pair<DD>(v[i], lo, hi);
        v[i] = med3_u32(lo, hi, cm);
      } else {
        v[i] = med3_u32(v[i], xch<DD>(v[i], addr), cm);
      }
    }
    return;
  }
  if constexpr (DD == 16 || DD == 32) {
    // the row swap yields both values of the lane pair: no partner select
#pragma unroll
    for (int i = 0; i < E; i++) {
      T lo, hi;
      swap_pair<DD>(v[i], lo, hi);
      const bool ol = R::less(hi, lo);
      const T mn = R::sel(ol, hi, lo), mx = R::sel(ol, lo, hi);
      v[i] = R::sel(take_min, mn, mx);
    }
    return;
  }
#pragma unroll
  for (int i0 = 0; i0 < E; i0 += GB) {
    T o[GB];
#pragma unroll
    for (int g = 0; g < GB; g++) o[g] = xch<DD>(v[i0 + g], addr);
#pragma unroll
    for (int g = 0; g < GB; g++) {
      const bool ol = R::less(o[g], v[i0 + g]);
      const T mn = R::sel(ol, o[g], v[i0 + g]), mx = R::sel(ol, v[i0 + g], o[g]);
      v[i0 + g] = R::sel(take_min, mn, mx);
    }
  }
}

// Write a sorted small part from LDS to K (and V).  The LDS reads are
// unconditional, eight at a time ahead of their stores, so they are in flight
// together rather than one read and wait per store: slots [len, NT*E) lie in
// the part's LDS area (NT*E is the part's padded power-of-two size) and are
// read but never stored; a payload is gathered only for a slot below len.
template <int DT, bool HASV, int NT, int E, bool DBG>
__device__ __attribute__((always_inline)) inline void write_part(
    const Ctx &c, const typename Rec<typename Codec<DT>::B, HASV>::T *lds, const uint32_t *srcV,
    typename Codec<DT>::B *K, uint64_t off, uint32_t len, uint32_t t) {
  using R = Rec<typename Codec<DT>::B, HASV>;
  constexpr int WB = E < 8 ? E : 8;
  // the thread index as an opaque value: the slot indices below are recomputed
  // per part instead of held in registers across parts
  uint32_t tv = t;
  opaque_v(tv);
  uint32_t pv[HASV ? E : 1];
  if constexpr (HASV) {
#pragma unroll
    for (int i = 0; i < E; i++) {
      const uint32_t x = (uint32_t)i * NT + tv;
      const uint32_t li = x < len ? R::idx(lds[lds_stripe<NT>(i, tv)]) : 0u;
      pv[i] = srcV[off + li];
    }
    group_sync<NT>();   // every payload is read before any is overwritten (in-place parts)
  }
#pragma unroll
  for (int i0 = 0; i0 < E; i0 += WB) {
    typename R::T o[WB];
#pragma unroll
    for (int g = 0; g < WB; g++) o[g] = lds[lds_stripe<NT>(i0 + g, tv)];
#pragma unroll
    for (int g = 0; g < WB; g++) {
      const uint32_t x = (uint32_t)(i0 + g) * NT + tv;
      if (x < len) {
        K[off + x] = Codec<DT>::dec(R::code(o[g]));
        if constexpr (HASV) c.V[off + x] = pv[i0 + g];
        if constexpr (DBG) dbg_final(c, off + x);
      }
    }
  }
}

// Sort one small part of len <= NT*E keys with NT threads (one wave or the whole
// workgroup), E consecutive elements per thread, and write it to K (and V).
template <int DT, bool HASV, int NT, int E, bool DBG>
__device__ void sort_group(const Ctx &c, const FinItem &it,
                           typename Rec<typename Codec<DT>::B, HASV>::T *lds, uint32_t t) {
  using B = typename Codec<DT>::B;
  using R = Rec<B, HASV>;
  using T = typename R::T;
  constexpr uint32_t P = (uint32_t)NT * E;
  const bool in_s = (it.kind & 2u) != 0;
  const B *src = (const B *)(in_s ? c.S : c.K);
  const uint32_t *srcV = in_s ? c.VS : c.V;
  B *K = (B *)c.K;
  const uint32_t len = it.len;
  const uint64_t off = it.off;
  const uint32_t lane = t & 63u;
  // coalesced load into LDS, then the blocked layout into registers; loads are
  // unconditional (index clamped into the part) and issued eight at a time so
  // they are in flight together
  constexpr int LB = E < 8 ? E : 8;
#pragma unroll
  for (int i0 = 0; i0 < E; i0 += LB) {
    B kin[LB];
#pragma unroll
    for (int g = 0; g < LB; g++) {
      const uint32_t x = (uint32_t)(i0 + g) * NT + t;
      kin[g] = src[off + (x < len ? x : len - 1)];
    }
#pragma unroll
    for (int g = 0; g < LB; g++) {
      const uint32_t x = (uint32_t)(i0 + g) * NT + t;
      lds[lds_pad(x)] = x < len ? R::make(Codec<DT>::enc(kin[g]), x) : R::pad();
    }
  }
  group_sync<NT>();
  T v[E];
#pragma unroll
  for (int i = 0; i < E; i++) v[i] = lds[lds_pad(t * E + i)];
  group_sync<NT>();
  sort_regs_asc<R, E>(v);
  reverse_if<R, E>(v, (t & 1u) != 0);
  for (uint32_t k = 2 * E; k <= P; k <<= 1) {
    const bool asc = ((t * E) & k) == 0;
    for (uint32_t j = k >> 1; j >= (uint32_t)E; j >>= 1) {
      const uint32_t dd = j / E;
      const bool take_min = ((t & dd) == 0) == asc;
      if (NT == kWave || dd < (uint32_t)kWave) {
        const int addr = (int)((lane ^ dd) << 2);
        switch (dd) {
          case 1: cross_stage<R, E, 1>(v, take_min, addr); break;
          case 2: cross_stage<R, E, 2>(v, take_min, addr); break;
          case 4: cross_stage<R, E, 4>(v, take_min, addr); break;
          case 8: cross_stage<R, E, 8>(v, take_min, addr); break;
          case 16: cross_stage<R, E, 16>(v, take_min, addr); break;
          case 32: cross_stage<R, E, 32>(v, take_min, addr); break;
          default: cross_stage<R, E, 0>(v, take_min, addr); break;
        }
      } else {
#pragma unroll
        for (int i = 0; i < E; i++) lds[lds_pad((uint32_t)i * NT + t)] = v[i];
        group_sync<NT>();
#pragma unroll
        for (int i = 0; i < E; i++) {
          const T o = lds[lds_pad((uint32_t)i * NT + (t ^ dd))];
          const bool ol = R::less(o, v[i]);
          const T mn = R::sel(ol, o, v[i]), mx = R::sel(ol, v[i], o);
          v[i] = R::sel(take_min, mn, mx);
        }
        group_sync<NT>();
      }
    }
    merge_regs_asc<R, E>(v);
    reverse_if<R, E>(v, !asc);
  }
#pragma unroll
  for (int i = 0; i < E; i++) lds[lds_pad(t * E + i)] = v[i];
  group_sync<NT>();
  write_part<DT, HASV, NT, E, DBG>(c, lds, srcV, K, off, len, t);
  if (c.req_left) __threadfence();
  group_sync<NT>();
  if (c.req_left && t == 0) req_final(c, it.kind >> 2, len);
}

// Length of the sorted runs the register phase of the merging sort leaves
// (cross-lane merging stops at a wave's records or at the padded part).
template <int NT, int E>
__device__ inline uint32_t hyb_run(uint32_t Lp) {
  uint32_t k = E;
  while (k < Lp && k < (uint32_t)kWave * E && k < (uint32_t)NT * E) k <<= 1;
  return k;
}

// Sort one small part of len <= NT*E keys with NT threads by merging: every
// thread sorts E consecutive records in registers (a sorting network), then
// runs of E, 2E, 4E, ... keys are merged pairwise in LDS.  For each merge a
// thread owns E consecutive outputs: it finds where they start on the merge
// path of its two runs (binary search along the cross diagonal), at A[ai] and
// B[bi].  Positions len..Lp-1 (Lp = len rounded up to E) hold padding records,
// which sort last.
//   REG = false: the outputs are produced in order, one LDS read per output
//   (each read waits for the previous comparison).
//   REG = true: the outputs are the E smallest of A[ai, ai+E) and B[bi, bi+E)
//   (padding past a run's end); the pairwise minima of A[ai+i] and
//   B[bi+E-1-i] are exactly those E records, in bitonic order (Batcher's
//   merge), and a half-cleaner network in registers sorts them: 2E independent
//   LDS reads per thread and no dependent chain.
template <int DT, bool HASV, int NT, int E, bool REG, bool HYB, bool DBG>
__device__ __attribute__((always_inline)) void merge_group(const Ctx &c, const FinItem &it,
                            typename Rec<typename Codec<DT>::B, HASV>::T *lds, uint32_t t) {
  using B = typename Codec<DT>::B;
  using R = Rec<B, HASV>;
  using T = typename R::T;
  const bool in_s = (it.kind & 2u) != 0;
  const B *src = (const B *)(in_s ? c.S : c.K);
  const uint32_t *srcV = in_s ? c.VS : c.V;
  B *K = (B *)c.K;
  const uint32_t len = it.len;
  const uint64_t off = it.off;
  const uint32_t Lp = (len + E - 1) / E * E;
  const bool act = t * (uint32_t)E < Lp;
  // coalesced load into LDS (unconditional loads, index clamped into the part,
  // issued eight at a time); the slot indices come from an opaque copy of the
  // thread index, recomputed per part rather than held across parts
  uint32_t tv = t;
  opaque_v(tv);
  constexpr int LB = E < 8 ? E : 8;
#pragma unroll
  for (int i0 = 0; i0 < E; i0 += LB) {
    B kin[LB];
#pragma unroll
    for (int g = 0; g < LB; g++) {
      const uint32_t x = (uint32_t)(i0 + g) * NT + tv;
      kin[g] = src[off + (x < len ? x : len - 1)];
    }
#pragma unroll
    for (int g = 0; g < LB; g++) {
      const uint32_t x = (uint32_t)(i0 + g) * NT + tv;
      if (x < Lp) lds[lds_stripe<NT>(i0 + g, tv)] = x < len ? R::make(Codec<DT>::enc(kin[g]), x) : R::pad();
    }
  }
  group_sync<NT>();
  T v[E];
  uint32_t r0 = E;   // sorted run length in LDS after the register phase
  if constexpr (HYB) {
    // runs of up to a wave's records are merged in registers by bitonic
    // cross-lane stages (lane exchanges, no LDS), the last round ascending
    // everywhere; records past Lp are padding.  A wave whose records all lie
    // past Lp has nothing to sort (the merges below read only [0, Lp)).
    const uint32_t kmax = hyb_run<NT, E>(Lp);
    r0 = kmax;
    if (NT == kWave || (t & ~(uint32_t)(kWave - 1)) * (uint32_t)E < Lp) {
#pragma unroll
      for (int i = 0; i < E; i++) v[i] = act ? lds[lds_pad(t * E + i)] : R::pad();
      sort_regs_asc<R, E>(v);
      if (kmax > (uint32_t)E) reverse_if<R, E>(v, (t & 1u) != 0);
      // round m merges runs of E << (m - 1) into runs of E << m: partners at
      // 2^(m-1), ..., 2, 1 lanes
      static_for<1, 7>([&](auto M) __attribute__((always_inline)) {
        constexpr int m = decltype(M)::value;
        const uint32_t k = (uint32_t)E << m;
        if (k <= kmax) {
          const bool asc = k == kmax || ((t * E) & k) == 0;
          // stage by stage: scheduling across stages only raises register pressure
          if constexpr (m >= 6) cross_stage<R, E, 32>(v, ((t & 32u) == 0) == asc, 0);
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (m >= 5) cross_stage<R, E, 16>(v, ((t & 16u) == 0) == asc, 0);
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (m >= 4) cross_stage<R, E, 8>(v, ((t & 8u) == 0) == asc, 0);
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (m >= 3) cross_stage<R, E, 4>(v, ((t & 4u) == 0) == asc, 0);
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (m >= 2) cross_stage<R, E, 2>(v, ((t & 2u) == 0) == asc, 0);
          __builtin_amdgcn_sched_barrier(0);
          cross_stage<R, E, 1>(v, ((t & 1u) == 0) == asc, 0);
          __builtin_amdgcn_sched_barrier(0);
          merge_regs_dir<R, E>(v, asc);
          __builtin_amdgcn_sched_barrier(0);
        }
      });
    }
  } else if (act) {
#pragma unroll
    for (int i = 0; i < E; i++) v[i] = lds[lds_pad(t * E + i)];
    sort_regs_asc<R, E>(v);
  }
  group_sync<NT>();
  if (act) {
#pragma unroll
    for (int i = 0; i < E; i++) lds[lds_pad(t * E + i)] = v[i];
  }
  for (uint32_t r = r0; r < Lp; r <<= 1) {
    group_sync<NT>();
    const uint32_t p0 = t * E;
    const uint32_t base = p0 & ~(2 * r - 1);
    const uint32_t diag = p0 - base;
    const uint32_t rA = Lp - base < r ? Lp - base : r;
    const uint32_t rB = Lp - base > r ? (Lp - base - r < r ? Lp - base - r : r) : 0u;
    if (act && rB > 0) {
      const uint32_t a0 = base, b0 = base + rA;
      // first diag outputs take lo records of A: the largest lo with
      // A[lo-1] <= B[diag-lo] (ties go to A)
      uint32_t lo = diag > rB ? diag - rB : 0u, hi = diag < rA ? diag : rA;
      while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (!R::less(lds[lds_pad(b0 + diag - 1 - m)], lds[lds_pad(a0 + m)])) lo = m + 1;
        else hi = m;
      }
      uint32_t ai = lo, bi = diag - lo;
      if constexpr (REG) {
#pragma unroll
        for (int i = 0; i < E; i++) {
          const uint32_t ia = ai + (uint32_t)i, ib = bi + (uint32_t)(E - 1 - i);
          const T xa = lds[lds_pad(a0 + (ia < rA ? ia : rA - 1))];
          const T xb = lds[lds_pad(b0 + (ib < rB ? ib : rB - 1))];
          const T pa = R::sel(ia < rA, xa, R::pad()), pb = R::sel(ib < rB, xb, R::pad());
          v[i] = R::sel(R::less(pb, pa), pb, pa);
        }
        merge_regs_asc<R, E>(v);
      } else {
        const uint32_t last = Lp - 1;
        T a = lds[lds_pad(a0 + (ai < rA ? ai : rA - 1))];
        T b = lds[lds_pad(b0 + (bi < rB ? bi : rB - 1))];
#pragma unroll
        for (int i = 0; i < E; i++) {
          const bool ta = bi >= rB || (ai < rA && !R::less(b, a));
          v[i] = R::sel(ta, a, b);
          ai += ta ? 1u : 0u;
          bi += ta ? 0u : 1u;
          uint32_t nx = ta ? a0 + ai : b0 + bi;
          nx = nx < last ? nx : last;
          const T y = lds[lds_pad(nx)];
          a = R::sel(ta, y, a);
          b = R::sel(ta, b, y);
        }
      }
    }
    group_sync<NT>();
    if (act && rB > 0) {
#pragma unroll
      for (int i = 0; i < E; i++) lds[lds_pad(t * E + i)] = v[i];
    }
  }
  group_sync<NT>();
  write_part<DT, HASV, NT, E, DBG>(c, lds, srcV, K, off, len, t);
  if (c.req_left) __threadfence();
  group_sync<NT>();
  if (c.req_left && t == 0) req_final(c, it.kind >> 2, len);
}

template <int DT, bool HASV, bool DBG = false>
__device__ inline void fill_band(const Ctx &c, const FinItem &it, uint32_t t, uint32_t nt) {
  using B = typename Codec<DT>::B;
  B *K = (B *)c.K;
  const B kv = Codec<DT>::dec((B)it.pivot);
  for (uint32_t q = t; q < it.len; q += nt) {
    K[it.off + q] = kv;
    if constexpr (HASV) c.V[it.off + q] = c.VE[it.src + q];
    if constexpr (DBG) dbg_final(c, it.off + q);
  }
}

// Level d's finishing work: long-band chunks and workgroup-sized small parts
// (workgroup each), then wave-sized small parts and short bands (wave each).
// Child slots are [0, 4 * parts of level d), band slots [0, 3 * parts); at the
// roots' level also the root slots.
// ALGO: 0 bitonic network, 1 merging with ordered outputs, 2 as 3 with
// register merge networks for the merges in LDS, 3 merging with ordered outputs
// after cross-lane bitonic merging of runs of up to a wave (merge_group).
// One small part sorted by a workgroup of NTW threads (the algorithm's
// records per thread chosen by the part's padded size).
template <int DT, bool HASV, int ALGO, int NTW, bool DBG>
__device__ __attribute__((always_inline)) inline void finish_group(
    const Ctx &c, const FinItem &it, typename Rec<typename Codec<DT>::B, HASV>::T *lds, uint32_t tid) {
  constexpr bool BITONIC = ALGO == 0, REG = ALGO == 2, HYB = ALGO >= 2;
  using T = typename Rec<typename Codec<DT>::B, HASV>::T;
  const uint32_t P = next_pow2(it.len);
  constexpr int ME = max_e<T>();
  if constexpr (BITONIC) {
    if (P <= 4 * NTW) sort_group<DT, HASV, NTW, 4, DBG>(c, it, lds, tid);
    else if (P <= 8 * NTW || ME < 16) sort_group<DT, HASV, NTW, 8, DBG>(c, it, lds, tid);
    else if constexpr (ME >= 16) {
      if (P <= 16 * NTW || ME < 32) sort_group<DT, HASV, NTW, 16, DBG>(c, it, lds, tid);
      else if constexpr (ME >= 32) sort_group<DT, HASV, NTW, 32, DBG>(c, it, lds, tid);
    }
  } else {
    if (P <= 4 * NTW) merge_group<DT, HASV, NTW, 4, REG, HYB, DBG>(c, it, lds, tid);
    else if (P <= 8 * NTW || ME < 16) merge_group<DT, HASV, NTW, 8, REG, HYB, DBG>(c, it, lds, tid);
    else if constexpr (ME >= 16) {
      if (P <= 16 * NTW || ME < 32) merge_group<DT, HASV, NTW, 16, REG, HYB, DBG>(c, it, lds, tid);
      else if constexpr (ME >= 32) merge_group<DT, HASV, NTW, 32, REG, HYB, DBG>(c, it, lds, tid);
    }
  }
}

// One small part of at most wave_max keys sorted by a wave.
template <int DT, bool HASV, int ALGO, bool DBG>
__device__ __attribute__((always_inline)) inline void finish_wave(
    const Ctx &c, const FinItem &it, typename Rec<typename Codec<DT>::B, HASV>::T *wl, uint32_t lane) {
  constexpr bool BITONIC = ALGO == 0, REG = ALGO == 2, HYB = ALGO >= 2;
  using T = typename Rec<typename Codec<DT>::B, HASV>::T;
  const uint32_t P = next_pow2(it.len);
  constexpr int ME = max_e<T>();
  if constexpr (BITONIC) {
    if (P <= 64) sort_group<DT, HASV, kWave, 1, DBG>(c, it, wl, lane);
    else if (P <= 128) sort_group<DT, HASV, kWave, 2, DBG>(c, it, wl, lane);
    else if (P <= 256) sort_group<DT, HASV, kWave, 4, DBG>(c, it, wl, lane);
    else if (P <= 512 || ME < 16) sort_group<DT, HASV, kWave, 8, DBG>(c, it, wl, lane);
    else if constexpr (ME >= 16) {
      if (P <= 1024 || ME < 32) sort_group<DT, HASV, kWave, 16, DBG>(c, it, wl, lane);
      else if constexpr (ME >= 32) sort_group<DT, HASV, kWave, 32, DBG>(c, it, wl, lane);
    }
  } else {
    if (P <= 64) merge_group<DT, HASV, kWave, 1, REG, HYB, DBG>(c, it, wl, lane);
    else if (P <= 128) merge_group<DT, HASV, kWave, 2, REG, HYB, DBG>(c, it, wl, lane);
    else if (P <= 256) merge_group<DT, HASV, kWave, 4, REG, HYB, DBG>(c, it, wl, lane);
    else if (P <= 512 || ME < 16) merge_group<DT, HASV, kWave, 8, REG, HYB, DBG>(c, it, wl, lane);
    else if constexpr (ME >= 16) {
      if (P <= 1024 || ME < 32) merge_group<DT, HASV, kWave, 16, REG, HYB, DBG>(c, it, wl, lane);
      else if constexpr (ME >= 32) merge_group<DT, HASV, kWave, 32, REG, HYB, DBG>(c, it, wl, lane);
    }
  }
}

template <int DT, bool HASV, int ALGO, bool DBG = false>
__global__ __launch_bounds__(kFinNT) __attribute__((amdgpu_waves_per_eu(4))) void k_finish(Ctx c, int d) {
  using B = typename Codec<DT>::B;
  using R = Rec<B, HASV>;
  using T = typename R::T;
  extern __shared__ unsigned char smem[];
  T *lds = reinterpret_cast<T *>(smem);
  const uint32_t nseg = (uint32_t)(c.lvl[d].packed >> 40);
  const uint32_t nbig = c.lvl[d].nbig;
  if (nseg > c.seg_cap || nbig > c.big_cap) return;
  const uint32_t nchild = c.fin_roots_only ? 0u : 4 * nseg;
  const uint32_t nbands = c.fin_roots_only ? 0u : 3 * nseg;
  const uint32_t nslots = nchild + (d == c.root_level ? c.nroots : 0u);
  const uint32_t tid = threadIdx.x;
  for (uint32_t ii = blockIdx.x; ii < nbig + nslots; ii += gridDim.x) {
    if (ii < nbig) {
      const FinItem bg = c.big[ii];
      fill_band<DT, HASV, DBG>(c, bg, tid, kFinNT);
      if (c.req_left) {
        __threadfence();
        __syncthreads();
        if (tid == 0) req_final(c, bg.kind >> 2, bg.len);
      }
      continue;
    }
    const uint32_t q = ii - nbig;
    const uint32_t slot = q < nchild ? q : 4 * c.seg_cap + (q - nchild);
    const FinItem it = c.fin[slot];
    if (it.len == 0) continue;
    finish_group<DT, HASV, ALGO, kFinNT, DBG>(c, it, lds, tid);
  }
  const uint32_t wv = tid / kWave, lane = tid & 63u;
  T *wl = lds + (size_t)wv * lds_pad(c.wave_max);
  const uint32_t gw = blockIdx.x * kFinNW + wv, nw = gridDim.x * kFinNW;
  for (uint32_t q = gw; q < nslots + nbands; q += nw) {
    if (q >= nslots) {
      const FinItem bd = c.band[q - nslots];
      if (bd.len) {
        fill_band<DT, HASV, DBG>(c, bd, lane, kWave);
        if (c.req_left) {
          __threadfence();
          __builtin_amdgcn_wave_barrier();
          if (lane == 0) req_final(c, bd.kind >> 2, bd.len);
        }
      }
      continue;
    }
    const uint32_t slot = q < nchild ? q : 4 * c.seg_cap + (q - nchild);
    const FinItem it = c.finw[slot];
    if (it.len == 0) continue;
    finish_wave<DT, HASV, ALGO, DBG>(c, it, wl, lane);
  }
}

// The small parts the persistent kernel listed (after it has ended).
template <int DT, bool HASV, int ALGO, bool DBG = false>
__global__ __launch_bounds__(kFinNT) __attribute__((amdgpu_waves_per_eu(4))) void k_finish_list(Ctx c) {
  using T = typename Rec<typename Codec<DT>::B, HASV>::T;
  extern __shared__ unsigned char smem[];
  T *lds = reinterpret_cast<T *>(smem);
  const unsigned long long nf = c.p.ctl[kQFin], nw = c.p.ctl[kQFinw];
  if (nf + nw > c.p.sfin_cap) return;   // overflow (reported by the persistent kernel)
  const uint32_t tid = threadIdx.x;
  for (unsigned long long i = blockIdx.x; i < nf; i += gridDim.x)
    finish_group<DT, HASV, ALGO, kFinNT, DBG>(c, c.p.sfin[i], lds, tid);
  const uint32_t wv = tid / kWave, lane = tid & 63u;
  T *wl = lds + (size_t)wv * lds_pad(c.wave_max);
  for (unsigned long long i = (unsigned long long)blockIdx.x * kFinNW + wv; i < nw;
       i += (unsigned long long)gridDim.x * kFinNW)
    finish_wave<DT, HASV, ALGO, DBG>(c, c.p.sfin[c.p.sfin_cap - 1 - i], wl, lane);
}

}  // namespace tsqs
