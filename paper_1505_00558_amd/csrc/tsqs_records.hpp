// tsqs_records.hpp -- records of any size sorted by their keys (late swapping, SVIII.H).
//
// The paper sorts an array of pointers to large elements and only then moves
// every element once into its final place.  Here the pointer array is a uint32
// index sorted as the payload of the keys; the move is a gather: output record i
// is input record index[i].  One thread copies one record, in words of the widest
// type that the record size and both buffers' alignment allow.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tsqs {

constexpr int kRecNT = 256;

__global__ __launch_bounds__(kRecNT) void k_rec_iota(uint32_t *idx, uint64_t n, unsigned int *err) {
  const uint64_t step = (uint64_t)gridDim.x * kRecNT;
  for (uint64_t i = (uint64_t)blockIdx.x * kRecNT + threadIdx.x; i < n; i += step) idx[i] = (uint32_t)i;
  if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0u;
}

constexpr int kRecU = 4;            // output words per thread per tile (loads in flight)

// dst[r] = src[idx[r]] for records of wpr words of type W.  The output is cut into
// tiles of kRecNT * kRecU consecutive words; thread t copies words t, t + kRecNT,
// ... of its tile, so every store is coalesced and the lanes that fall in one
// record read that record's consecutive words.  An index out of range (not a
// permutation: a bug) is reported in *err instead of being followed.
template <typename W>
__global__ __launch_bounds__(kRecNT) void k_rec_gather(const W *__restrict__ src, W *__restrict__ dst,
                                                      const uint32_t *__restrict__ idx, uint64_t n,
                                                      uint32_t wpr, unsigned int *err) {
  const uint64_t total = n * wpr;
  const uint64_t tile_words = (uint64_t)kRecNT * kRecU;
  const uint64_t tiles = (total + tile_words - 1) / tile_words;
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const uint64_t tb = t * tile_words;
    const uint64_t r0 = tb / wpr;                       // record of the tile's first word
    const uint32_t lw0 = (uint32_t)(tb - r0 * wpr);     // its word within that record
    uint64_t w[kRecU], s[kRecU];
    bool ok[kRecU];
#pragma unroll
    for (int u = 0; u < kRecU; u++) {
      w[u] = tb + (uint64_t)u * kRecNT + threadIdx.x;
      const uint32_t lw = lw0 + (uint32_t)u * kRecNT + threadIdx.x;
      const uint32_t lr = lw / wpr;
      const uint64_t r = r0 + lr;
      ok[u] = w[u] < total;
      const uint32_t k = ok[u] ? idx[r] : 0u;
      if (ok[u] && k >= n) { atomicOr(err, 1u); ok[u] = false; }
      s[u] = (uint64_t)k * wpr + (lw - lr * wpr);
    }
    W v[kRecU];
#pragma unroll
    for (int u = 0; u < kRecU; u++)
      if (ok[u]) v[u] = src[s[u]];
#pragma unroll
    for (int u = 0; u < kRecU; u++)
      if (ok[u]) dst[w[u]] = v[u];
  }
}

}  // namespace tsqs
