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

// dst[r] = src[idx[r]] for records of wpr words of type W; an index out of range
// (not a permutation: a bug) is reported in *err instead of being followed.
template <typename W>
__global__ __launch_bounds__(kRecNT) void k_rec_gather(const W *__restrict__ src, W *__restrict__ dst,
                                                      const uint32_t *__restrict__ idx, uint64_t n,
                                                      uint32_t wpr, unsigned int *err) {
  const uint64_t step = (uint64_t)gridDim.x * kRecNT;
  for (uint64_t r = (uint64_t)blockIdx.x * kRecNT + threadIdx.x; r < n; r += step) {
    const uint32_t k = idx[r];
    if (k >= n) { atomicOr(err, 1u); continue; }
    const W *s = src + (uint64_t)k * wpr;
    W *d = dst + r * wpr;
    for (uint32_t j = 0; j < wpr; j++) d[j] = s[j];
  }
}

}  // namespace tsqs
