// tsqs_kernels.hpp -- gfx950 kernels of the three-way partition sort.
//
// The method is the recursion of Triple State QuickSort (Muqaddas, arXiv
// 1505.00558, SIII): pick a pivot from samples, split a part into keys < p,
// keys == p and keys > p, put the == p keys in a middle band that is final and
// never compared again, recurse on the two sides.  The paper's single-threaded
// hole-juggling scan (SIII.A-F) is not used; on the GPU one level of the
// recursion is one data-parallel pass over every active part:
//
//   k_partition  every 4096-key tile of every part at this level: coalesced
//                loads, two compares per key on an order-preserving unsigned
//                code, ranks from 64-lane ballots + mbcnt, an LDS prefix over
//                (item, wave), ONE packed 64-bit atomic per tile reserving
//                [left cursor, right cursor] in the part, and stores of the
//                < and > keys into the other buffer (ping-pong K <-> S).
//   k_plan       one workgroup per part just partitioned: reads the final
//                cursors, emits the equal band, and for each child either a
//                small-part item or a part of the next level with a pivot
//                (median of up to 63 samples sorted inside one wave; the exact
//                median by radix select once the depth limit is reached).
//   k_finish     one workgroup per item: small parts are sorted in LDS by a
//                bitonic network and written to K; band chunks write the pivot
//                value (equality means identical bits) and the staged payloads.
//
// Buffers: a part at depth d lives in K when d is even, in S when d is odd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsqs {

constexpr int kWave = 64;
constexpr int kPartWG = 256;
constexpr int kPartWaves = kPartWG / kWave;
constexpr int kIPT = 16;                        // keys per thread per tile
constexpr uint32_t kTile = kPartWG * kIPT;      // 4096 keys per tile
static_assert(kIPT * kPartWaves == kWave, "one wave scans the (item, wave) counts");
constexpr int kPlanWG = 256;
constexpr int kFinWG = 256;
constexpr uint32_t kBandChunk = 1u << 16;
constexpr int kMaxLevels = 192;
constexpr unsigned long long kTileMask = (1ull << 40) - 1;
constexpr uint32_t kErrSegCap = 1, kErrFinCap = 2, kErrLevel = 4;

// ---- order-preserving codes (compares are done on these, never on floats) --

template <int DT> struct Codec;
template <> struct Codec<0> {  // int32: flip the sign bit
  using B = uint32_t;
  __device__ static inline B enc(B x) { return x ^ 0x80000000u; }
  __device__ static inline B dec(B u) { return u ^ 0x80000000u; }
};
template <> struct Codec<1> {  // uint32
  using B = uint32_t;
  __device__ static inline B enc(B x) { return x; }
  __device__ static inline B dec(B u) { return u; }
};
template <> struct Codec<2> {  // int64
  using B = uint64_t;
  __device__ static inline B enc(B x) { return x ^ 0x8000000000000000ull; }
  __device__ static inline B dec(B u) { return u ^ 0x8000000000000000ull; }
};
template <> struct Codec<3> {  // uint64
  using B = uint64_t;
  __device__ static inline B enc(B x) { return x; }
  __device__ static inline B dec(B u) { return u; }
};
template <> struct Codec<4> {  // float32 bits, IEEE totalOrder: negatives reversed
  using B = uint32_t;
  __device__ static inline B enc(B x) {
    return x ^ ((uint32_t)((int32_t)x >> 31) | 0x80000000u);
  }
  __device__ static inline B dec(B u) {
    return u ^ (~(uint32_t)((int32_t)u >> 31) | 0x80000000u);
  }
};

// ---- device tables -----------------------------------------------------------

struct Seg {                 // one part of a level
  uint64_t off;              // first key
  uint64_t pivot;            // encoded pivot
  uint32_t len;
  uint32_t tile_begin;       // first tile of this part in the level's tile space
  uint32_t depth;
  uint32_t dmax;             // depth limit of the array it came from
};

struct FinItem {             // work of the finish kernel
  uint64_t off;              // small part: first key; band chunk: first band slot
  uint64_t src;              // band chunk: first staged payload in VE
  uint64_t pivot;            // band chunk: encoded key of the band
  uint32_t len;
  uint32_t kind;             // bit 0: band chunk; bit 1: small part lives in S
};

struct LevelCtl {
  unsigned long long packed; // parts << 40 | tiles of this level
  unsigned long long keys;   // keys in the parts of this level
  unsigned int nfin;         // finish items emitted at this level
  unsigned int pad0;
  unsigned long long pad1;
};

struct DevStats {
  unsigned long long fallback_parts, small_parts, small_keys, band_keys;
  unsigned int max_depth, err;
};

struct Ctx {
  void *K, *S;
  uint32_t *V, *VS, *VE;
  Seg *seg0, *seg1;
  unsigned long long *ctr0, *ctr1;   // packed (left count | right count << 32)
  unsigned int *ectr0, *ectr1;       // equal-key count (payload staging)
  FinItem *fin;
  LevelCtl *lvl;
  DevStats *st;
  const uint64_t *roots;             // nroots+1 offsets, or null: one root [0, n)
  uint64_t n;
  uint32_t nroots;
  uint32_t small_max;
  uint32_t samples;
  uint32_t depth_factor;
  uint32_t pivot_mode;               // 0 sampled median, 1 exact minimum
  uint32_t jitter;                   // per-call sample shift
  uint32_t seg_cap;
  uint32_t fin_cap;
};

// ---- wave helpers ------------------------------------------------------------

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of m in lanes below this one
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

// ---- pivot choice ----------------------------------------------------------------

// Median of S samples (S odd, <= 63) at evenly spaced positions of Y[off, off+len);
// interior samples (not the first, middle or last) are shifted toward the middle
// or away from it by a per-call amount of at most a quarter spacing (the paper's
// sample jitter against crafted inputs, SV.C).  Run by one whole wave.
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

// Exact k-th smallest code of Y[off, off+len) by most-significant-digit radix
// select (8-bit digits, 256-bin LDS histograms).  Whole workgroup, read-only.
template <int DT, int NT>
__device__ typename Codec<DT>::B wg_select(const typename Codec<DT>::B *Y, uint64_t off,
                                           uint32_t len, uint32_t k, uint32_t *hist,
                                           unsigned long long *bcast) {
  using B = typename Codec<DT>::B;
  constexpr int BITS = (int)sizeof(B) * 8;
  B prefix = 0, mask = 0;
  uint32_t krem = k;
  for (int shift = BITS - 8; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < len; i += NT) {
      B u = Codec<DT>::enc(Y[off + i]);
      if ((u & mask) == prefix) atomicAdd(&hist[(uint32_t)(u >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0, sel = 255;
      for (uint32_t dgt = 0; dgt < 256; dgt++) {
        if (acc + hist[dgt] > krem) { sel = dgt; break; }
        acc += hist[dgt];
      }
      bcast[0] = (unsigned long long)(prefix | ((B)sel << shift));
      bcast[1] = krem - acc;
    }
    __syncthreads();
    prefix = (B)bcast[0];
    krem = (uint32_t)bcast[1];
    mask |= (B)255 << shift;
    __syncthreads();
  }
  return prefix;
}

// Pivot of a part, computed by the whole workgroup (result in every thread).
template <int DT>
__device__ typename Codec<DT>::B choose_pivot(const Ctx &c, const typename Codec<DT>::B *Y,
                                              uint64_t off, uint32_t len, uint32_t depth,
                                              uint32_t dmax, uint32_t *hist,
                                              unsigned long long *bcast) {
  using B = typename Codec<DT>::B;
  if (c.pivot_mode == 1 || depth >= dmax) {
    uint32_t k = (c.pivot_mode == 1 && depth < dmax) ? 0u : len / 2;
    if (threadIdx.x == 0 && depth >= dmax) atomicAdd(&c.st->fallback_parts, 1ull);
    return wg_select<DT, kPlanWG>(Y, off, len, k, hist, bcast);
  }
  if (threadIdx.x < kWave) {
    uint32_t S = c.samples;
    if (S > len) S = (len & 1) ? len : len - 1;
    B p = wave_sample_pivot<DT>(Y, off, len, S, c.jitter);
    if (threadIdx.x == 0) bcast[2] = (unsigned long long)p;
  }
  __syncthreads();
  B p = (B)bcast[2];
  __syncthreads();
  return p;
}

// ---- emission (single thread) ---------------------------------------------------

template <bool HASV>
__device__ inline void emit_part(const Ctx &c, int lvl_next, uint64_t off, uint32_t len,
                                 uint64_t pivot, uint32_t depth, uint32_t dmax) {
  if (lvl_next >= kMaxLevels) { atomicOr(&c.st->err, kErrLevel); return; }
  const uint32_t tiles = (len + kTile - 1) / kTile;
  unsigned long long old = atomicAdd(&c.lvl[lvl_next].packed, (1ull << 40) | (unsigned long long)tiles);
  const uint32_t idx = (uint32_t)(old >> 40);
  if (idx >= c.seg_cap) { atomicOr(&c.st->err, kErrSegCap); return; }
  Seg s;
  s.off = off; s.pivot = pivot; s.len = len; s.tile_begin = (uint32_t)(old & kTileMask);
  s.depth = depth; s.dmax = dmax;
  Seg *segs = (lvl_next & 1) ? c.seg1 : c.seg0;
  segs[idx] = s;
  ((lvl_next & 1) ? c.ctr1 : c.ctr0)[idx] = 0ull;
  if (HASV) ((lvl_next & 1) ? c.ectr1 : c.ectr0)[idx] = 0u;
  atomicAdd(&c.lvl[lvl_next].keys, (unsigned long long)len);
  atomicMax(&c.st->max_depth, depth);
}

__device__ inline void emit_small(const Ctx &c, int level, uint64_t off, uint32_t len, bool in_s) {
  uint32_t i = atomicAdd(&c.lvl[level].nfin, 1u);
  if (i >= c.fin_cap) { atomicOr(&c.st->err, kErrFinCap); return; }
  FinItem it;
  it.off = off; it.src = 0; it.pivot = 0; it.len = len; it.kind = in_s ? 2u : 0u;
  c.fin[i] = it;
  atomicAdd(&c.st->small_parts, 1ull);
  atomicAdd(&c.st->small_keys, (unsigned long long)len);
}

__device__ inline void emit_band(const Ctx &c, int level, uint64_t off, uint64_t src,
                                 uint32_t len, uint64_t pivot) {
  const uint32_t nch = (len + kBandChunk - 1) / kBandChunk;
  uint32_t i0 = atomicAdd(&c.lvl[level].nfin, nch);
  if (i0 + nch > c.fin_cap) { atomicOr(&c.st->err, kErrFinCap); return; }
  for (uint32_t q = 0; q < nch; q++) {
    FinItem it;
    uint32_t base = q * kBandChunk;
    it.off = off + base; it.src = src + base; it.pivot = pivot;
    it.len = (len - base < kBandChunk) ? (len - base) : kBandChunk;
    it.kind = 1u;
    c.fin[i0 + q] = it;
  }
  atomicAdd(&c.st->band_keys, (unsigned long long)len);
}

// A child part of depth `depth` living in the buffer of that depth's parity:
// small -> finish item of level `fin_level`; large -> part of level
// `part_level` with its pivot.
template <int DT, bool HASV>
__device__ void handle_child(const Ctx &c, int fin_level, int part_level, uint64_t off,
                             uint32_t len, uint32_t depth, uint32_t dmax, uint32_t *hist,
                             unsigned long long *bcast) {
  using B = typename Codec<DT>::B;
  const bool in_s = (depth & 1) != 0;
  if (len == 0) return;
  if (len <= c.small_max) {
    if (threadIdx.x == 0 && (len > 1 || in_s)) emit_small(c, fin_level, off, len, in_s);
    return;
  }
  const B *Y = (const B *)(in_s ? c.S : c.K);
  B p = choose_pivot<DT>(c, Y, off, len, depth, dmax, hist, bcast);
  if (threadIdx.x == 0) emit_part<HASV>(c, part_level, off, len, (uint64_t)p, depth, dmax);
}

// ---- kernels ------------------------------------------------------------------------

__global__ void k_reset(Ctx c) {
  for (int i = threadIdx.x; i < kMaxLevels; i += blockDim.x) {
    c.lvl[i].packed = 0ull; c.lvl[i].keys = 0ull; c.lvl[i].nfin = 0u;
  }
  if (threadIdx.x == 0) {
    c.st->fallback_parts = 0; c.st->small_parts = 0; c.st->small_keys = 0;
    c.st->band_keys = 0; c.st->max_depth = 0; c.st->err = 0;
  }
}

// Roots: one workgroup per array.  A root is depth 0 and lives in K.
template <int DT, bool HASV>
__global__ __launch_bounds__(kPlanWG) void k_init(Ctx c) {
  __shared__ uint32_t hist[256];
  __shared__ unsigned long long bcast[4];
  for (uint32_t j = blockIdx.x; j < c.nroots; j += gridDim.x) {
    const uint64_t off = c.roots ? c.roots[j] : 0ull;
    const uint64_t end = c.roots ? c.roots[j + 1] : c.n;
    const uint32_t len = (uint32_t)(end - off);
    uint32_t lg = 0;
    while (lg < 32 && (1ull << lg) < (unsigned long long)len) lg++;
    const uint32_t dmax = c.depth_factor * lg;
    handle_child<DT, HASV>(c, 0, 0, off, len, 0u, dmax, hist, bcast);
  }
}

// One partition level: every tile of every part of level d.
template <int DT, bool HASV>
__global__ __launch_bounds__(kPartWG) void k_partition(Ctx c, int d) {
  using B = typename Codec<DT>::B;
  __shared__ uint32_t cntL[kWave], cntG[kWave], cntE[kWave];
  __shared__ uint32_t sh_seg;
  __shared__ unsigned long long sh_base;
  __shared__ uint32_t sh_baseE, sh_totG;

  const unsigned long long packed = c.lvl[d].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  const uint32_t ntiles = (uint32_t)(packed & kTileMask);
  // a failed capacity check leaves the count above the records written: stop
  if (ntiles == 0 || nseg > c.seg_cap) return;
  const Seg *segs = (d & 1) ? c.seg1 : c.seg0;
  unsigned long long *ctr = (d & 1) ? c.ctr1 : c.ctr0;
  unsigned int *ectr = (d & 1) ? c.ectr1 : c.ectr0;
  const B *X = (const B *)((d & 1) ? c.S : c.K);
  B *Y = (B *)((d & 1) ? c.K : c.S);
  const uint32_t *VX = (d & 1) ? c.VS : c.V;
  uint32_t *VY = (d & 1) ? c.V : c.VS;

  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;

  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    if (tid == 0) {
      uint32_t lo = 0, hi = nseg;
      while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (segs[mid].tile_begin <= t) lo = mid; else hi = mid;
      }
      sh_seg = lo;
    }
    __syncthreads();
    const Seg s = segs[sh_seg];
    const uint64_t tstart = s.off + (uint64_t)(t - s.tile_begin) * kTile;
    const uint64_t segend = s.off + s.len;
    const uint32_t cnt = (uint32_t)((segend - tstart) < kTile ? (segend - tstart) : kTile);
    const B pv = (B)s.pivot;

    B key[kIPT];
    uint32_t val[kIPT];
    uint32_t ltm = 0, gtm = 0, eqm = 0;
#pragma unroll
    for (int j = 0; j < kIPT; j++) {
      const uint32_t idx = (uint32_t)j * kPartWG + tid;
      const bool valid = idx < cnt;
      key[j] = valid ? X[tstart + idx] : (B)0;
      if (HASV) val[j] = valid ? VX[tstart + idx] : 0u;
      const B u = Codec<DT>::enc(key[j]);
      const bool lt = valid && (u < pv);
      const bool gt = valid && (u > pv);
      ltm |= (uint32_t)lt << j;
      gtm |= (uint32_t)gt << j;
      if (HASV) eqm |= (uint32_t)(valid && !lt && !gt) << j;
      const unsigned long long bl = __ballot(lt);
      const unsigned long long bg = __ballot(gt);
      if (lane == 0) {
        cntL[j * kPartWaves + w] = (uint32_t)__popcll(bl);
        cntG[j * kPartWaves + w] = (uint32_t)__popcll(bg);
      }
      if (HASV) {
        const unsigned long long be = __ballot(valid && !lt && !gt);
        if (lane == 0) cntE[j * kPartWaves + w] = (uint32_t)__popcll(be);
      }
    }
    __syncthreads();
    if (w == 0) {
      const uint32_t a = cntL[lane], b = cntG[lane];
      const uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
      uint32_t e = 0, ie = 0;
      if (HASV) { e = cntE[lane]; ie = wave_incl_scan(e); }
      if (lane == 63) {
        unsigned long long old = atomicAdd(&ctr[sh_seg], ((unsigned long long)ib << 32) | ia);
        sh_base = old;
        sh_totG = ib;
        if (HASV) sh_baseE = atomicAdd(&ectr[sh_seg], ie);
      }
      cntL[lane] = ia - a;
      cntG[lane] = ib - b;
      if (HASV) cntE[lane] = ie - e;
    }
    __syncthreads();
    const uint32_t baseL = (uint32_t)sh_base;
    const uint32_t baseG = (uint32_t)(sh_base >> 32);
    const uint64_t leftBase = s.off + baseL;
    const uint64_t rightBase = segend - baseG - sh_totG;
#pragma unroll
    for (int j = 0; j < kIPT; j++) {
      const bool lt = (ltm >> j) & 1u, gt = (gtm >> j) & 1u;
      const unsigned long long bl = __ballot(lt);
      const unsigned long long bg = __ballot(gt);
      if (lt) {
        const uint64_t pos = leftBase + cntL[j * kPartWaves + w] + mbcnt(bl);
        Y[pos] = key[j];
        if (HASV) VY[pos] = val[j];
      }
      if (gt) {
        const uint64_t pos = rightBase + cntG[j * kPartWaves + w] + mbcnt(bg);
        Y[pos] = key[j];
        if (HASV) VY[pos] = val[j];
      }
      if (HASV) {
        const bool eq = (eqm >> j) & 1u;
        const unsigned long long be = __ballot(eq);
        if (eq) c.VE[s.off + sh_baseE + cntE[j * kPartWaves + w] + mbcnt(be)] = val[j];
      }
    }
    __syncthreads();
  }
}

// After level d: bands, small children, next-level parts with pivots.
template <int DT, bool HASV>
__global__ __launch_bounds__(kPlanWG) void k_plan(Ctx c, int d) {
  __shared__ uint32_t hist[256];
  __shared__ unsigned long long bcast[4];
  const unsigned long long packed = c.lvl[d].packed;
  const uint32_t nseg = (uint32_t)(packed >> 40);
  if (nseg > c.seg_cap) return;
  const Seg *segs = (d & 1) ? c.seg1 : c.seg0;
  const unsigned long long *ctr = (d & 1) ? c.ctr1 : c.ctr0;
  for (uint32_t si = blockIdx.x; si < nseg; si += gridDim.x) {
    const Seg s = segs[si];
    const unsigned long long cv = ctr[si];
    const uint32_t L = (uint32_t)cv, G = (uint32_t)(cv >> 32);
    const uint32_t E = s.len - L - G;
    if (threadIdx.x == 0 && E > 0) emit_band(c, d, s.off + L, s.off, E, s.pivot);
    handle_child<DT, HASV>(c, d, d + 1, s.off, L, s.depth + 1, s.dmax, hist, bcast);
    handle_child<DT, HASV>(c, d, d + 1, s.off + s.len - G, G, s.depth + 1, s.dmax, hist, bcast);
  }
}

// LDS records of the small-part sort: the code, plus (with payloads) the local
// index, so that padding sorts after every real key and payloads can follow.
template <typename B, bool HASV> struct Rec;
template <typename B> struct Rec<B, false> {
  using T = B;
  __device__ static inline T make(B code, uint32_t) { return code; }
  __device__ static inline T pad() { return ~(B)0; }
  __device__ static inline B code(T r) { return r; }
  __device__ static inline bool less(T a, T b) { return a < b; }
};
template <> struct Rec<uint32_t, true> {
  using T = uint64_t;
  __device__ static inline T make(uint32_t code, uint32_t i) { return ((uint64_t)code << 32) | i; }
  __device__ static inline T pad() { return ~0ull; }
  __device__ static inline uint32_t code(T r) { return (uint32_t)(r >> 32); }
  __device__ static inline uint32_t idx(T r) { return (uint32_t)r; }
  __device__ static inline T with_idx(T r, uint32_t v) { return (r & 0xFFFFFFFF00000000ull) | v; }
  __device__ static inline bool less(T a, T b) { return a < b; }
};
struct R64 { uint64_t k; uint64_t i; };
template <> struct Rec<uint64_t, true> {
  using T = R64;
  __device__ static inline T make(uint64_t code, uint32_t i) { T r; r.k = code; r.i = i; return r; }
  __device__ static inline T pad() { T r; r.k = ~0ull; r.i = ~0ull; return r; }
  __device__ static inline uint64_t code(T r) { return r.k; }
  __device__ static inline uint32_t idx(T r) { return (uint32_t)r.i; }
  __device__ static inline T with_idx(T r, uint32_t v) { r.i = v; return r; }
  __device__ static inline bool less(T a, T b) { return a.k < b.k || (a.k == b.k && a.i < b.i); }
};

template <typename R>
__device__ void bitonic_lds(typename R::T *a, uint32_t P) {
  using T = typename R::T;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < P / 2; i += blockDim.x) {
        const uint32_t lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const uint32_t hi = lo + j;
        const bool up = (lo & k) == 0;
        T x = a[lo], y = a[hi];
        if (R::less(y, x) == up) { a[lo] = y; a[hi] = x; }
      }
      __syncthreads();
    }
  }
}

template <int DT, bool HASV>
__global__ __launch_bounds__(kFinWG) void k_finish(Ctx c, int d) {
  using B = typename Codec<DT>::B;
  using R = Rec<B, HASV>;
  using T = typename R::T;
  extern __shared__ unsigned char smem[];
  T *rec = reinterpret_cast<T *>(smem);
  const uint32_t nfin = c.lvl[d].nfin;
  if (nfin > c.fin_cap) return;
  B *K = (B *)c.K;
  for (uint32_t ii = blockIdx.x; ii < nfin; ii += gridDim.x) {
    const FinItem it = c.fin[ii];
    if (it.kind & 1u) {
      const B kv = Codec<DT>::dec((B)it.pivot);
      for (uint32_t q = threadIdx.x; q < it.len; q += kFinWG) {
        K[it.off + q] = kv;
        if (HASV) c.V[it.off + q] = c.VE[it.src + q];
      }
      continue;   // no LDS use, no barrier needed
    }
    const bool in_s = (it.kind & 2u) != 0;
    const B *src = in_s ? (const B *)c.S : (const B *)c.K;
    const uint32_t *srcV = in_s ? c.VS : c.V;
    uint32_t P = 1;
    while (P < it.len) P <<= 1;
    for (uint32_t q = threadIdx.x; q < P; q += kFinWG)
      rec[q] = q < it.len ? R::make(Codec<DT>::enc(src[it.off + q]), q) : R::pad();
    __syncthreads();
    bitonic_lds<R>(rec, P);
    if constexpr (HASV) {
      for (uint32_t q = threadIdx.x; q < it.len; q += kFinWG)
        rec[q] = R::with_idx(rec[q], srcV[it.off + R::idx(rec[q])]);
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < it.len; q += kFinWG) {
        K[it.off + q] = Codec<DT>::dec(R::code(rec[q]));
        c.V[it.off + q] = R::idx(rec[q]);
      }
    } else {
      for (uint32_t q = threadIdx.x; q < it.len; q += kFinWG)
        K[it.off + q] = Codec<DT>::dec(R::code(rec[q]));
    }
    __syncthreads();
  }
}

}  // namespace tsqs
