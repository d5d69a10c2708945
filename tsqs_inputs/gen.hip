// gen.hip -- device-side generator of the seeded synthetic inputs.
//
// Produces, in device memory, exactly the arrays that tsqs_inputs/__init__.py
// defines with numpy (same SplitMix64 stream, same families, same casts), so
// that inputs of tens of GB need not be generated on the host.  It holds no
// part of any sort.
//
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014):
//   x_i = mix(seed + (i + 1) * 0x9E3779B97F4A7C15),
//   mix(z) = z ^= z >> 30, z *= 0xBF58476D1CE4E5B9, z ^= z >> 27,
//            z *= 0x94D049BB133111EB, z ^= z >> 31.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

enum { F_UNIFORM = 0, F_SORTED, F_REVERSED, F_NEARLY, F_MANY_EQ, F_STAIR, F_ORGAN };
enum { D_I32 = 0, D_U32 = 1, D_I64 = 2, D_U64 = 3, D_F32 = 4 };

__device__ __host__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline uint64_t sm64(uint64_t seed, uint64_t i) {
  return mix64(seed + (i + 1) * 0x9E3779B97F4A7C15ull);
}

__device__ inline float normal_f32(uint64_t x) {
  const double u1 = ((double)(x >> 40) + 1.0) * 0x1p-24;
  const double u2 = (double)(x & 0xFFFFFFull) * 0x1p-24;
  return (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2));
}

__device__ inline uint32_t special_f32(uint64_t seed, uint64_t i) {
  const uint32_t bits[5] = {0x80000000u, 0x00000000u, 0x7F800000u, 0xFF800000u, 0x7FC00000u};
  const uint64_t sel = sm64(seed + 1, i) % 1000ull;
  if (sel < 5) return bits[sel];
  const float f = normal_f32(sm64(seed, i));
  return __float_as_uint(f);
}

__device__ inline int64_t index_value(int fam, uint64_t i, uint64_t n, uint64_t seed) {
  switch (fam) {
    case F_SORTED: case F_NEARLY: return (int64_t)i;
    case F_REVERSED: return (int64_t)(n - 1 - i);
    case F_MANY_EQ: return (int64_t)(sm64(seed, i) % 100ull);
    case F_STAIR: return (int64_t)(i / 1000);
    default: {  // organ pipe
      const uint64_t h = n / 2;
      return i < h ? (int64_t)(i + 1) : (int64_t)(n - i);
    }
  }
}

// One array element: value of family fam at index i of an n-element array.
__device__ inline void put(void *out, uint64_t at, int dt, int fam, uint64_t i, uint64_t n,
                           uint64_t seed) {
  if (fam == F_UNIFORM) {
    if (dt == D_F32) {
      ((uint32_t *)out)[at] = special_f32(seed, i);
    } else {
      const uint64_t x = sm64(seed, i);
      if (dt == D_I32 || dt == D_U32) ((uint32_t *)out)[at] = (uint32_t)x;
      else ((uint64_t *)out)[at] = x;
    }
    return;
  }
  const int64_t v = index_value(fam, i, n, seed);
  switch (dt) {
    case D_I32: case D_U32: ((uint32_t *)out)[at] = (uint32_t)v; break;
    case D_F32: ((float *)out)[at] = (float)v; break;
    default: ((uint64_t *)out)[at] = (uint64_t)v; break;
  }
}

struct Piece {       // a run of at most kPiece elements of one array
  uint64_t at;       // first output element
  uint64_t i0;       // its index within the array
  uint32_t arr;      // array number
  uint32_t cnt;      // elements in the piece
};

__global__ void k_fill(void *out, int dt, const Piece *pieces, const uint64_t *offs,
                       const int32_t *fams, const uint64_t *seeds) {
  const Piece p = pieces[blockIdx.x];
  const uint64_t n = offs[p.arr + 1] - offs[p.arr];
  const int fam = fams[p.arr];
  const uint64_t seed = seeds[p.arr];
  for (uint32_t k = threadIdx.x; k < p.cnt; k += blockDim.x)
    put(out, p.at + k, dt, fam, p.i0 + k, n, seed);
}

// nearly sorted: n / 200 swaps of positions (x_{2j} mod n, x_{2j+1} mod n),
// applied in order (one thread per array; later swaps may undo earlier ones)
__global__ void k_swaps(void *out, int dt, const uint64_t *offs, const int32_t *fams,
                        const uint64_t *seeds, uint32_t count) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= count || fams[a] != F_NEARLY) return;
  const uint64_t base = offs[a], n = offs[a + 1] - offs[a], seed = seeds[a];
  const uint64_t nsw = n / 200;
  if (n < 2) return;
  for (uint64_t j = 0; j < nsw; j++) {
    const uint64_t p = base + sm64(seed, 2 * j) % n, q = base + sm64(seed, 2 * j + 1) % n;
    if (dt == D_I64 || dt == D_U64) {
      uint64_t *o = (uint64_t *)out;
      const uint64_t t = o[p]; o[p] = o[q]; o[q] = t;
    } else {
      uint32_t *o = (uint32_t *)out;
      const uint32_t t = o[p]; o[p] = o[q]; o[q] = t;
    }
  }
}

constexpr uint32_t kPiece = 1u << 16;

}  // namespace

extern "C" {

// Fill d_out with `count` arrays laid back to back: array j occupies
// [h_offs[j], h_offs[j+1]) and holds family h_fams[j] (0 uniform, 1 sorted,
// 2 reversed, 3 nearly sorted, 4 many equals, 5 stair steps, 6 organ pipe)
// generated from seed h_seeds[j]; dt: 0 int32, 1 uint32, 2 int64, 3 uint64,
// 4 float32.  Host arrays; the call returns after the work is done.
// Returns 0, or -1 for bad arguments, -3 for a HIP error.
int tsqs_inputs_generate(void *d_out, int dt, const uint64_t *h_offs, const int32_t *h_fams,
                         const uint64_t *h_seeds, uint32_t count, void *stream) {
  if (!d_out || !h_offs || !h_fams || !h_seeds || dt < 0 || dt > 4) return -1;
  if (count == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  uint64_t npieces = 0;
  for (uint32_t j = 0; j < count; j++) {
    if (h_offs[j + 1] < h_offs[j]) return -1;
    if (h_fams[j] < 0 || h_fams[j] > 6) return -1;
    npieces += (h_offs[j + 1] - h_offs[j] + kPiece - 1) / kPiece;
  }
  if (npieces > 0x7FFFFFFFull) return -1;
  Piece *hp = (Piece *)malloc(sizeof(Piece) * (npieces ? npieces : 1));
  if (!hp) return -1;
  uint64_t k = 0;
  for (uint32_t j = 0; j < count; j++) {
    const uint64_t n = h_offs[j + 1] - h_offs[j];
    for (uint64_t i0 = 0; i0 < n; i0 += kPiece) {
      const uint64_t c = n - i0 < kPiece ? n - i0 : kPiece;
      hp[k++] = Piece{h_offs[j] + i0, i0, j, (uint32_t)c};
    }
  }
  Piece *dp = nullptr;
  uint64_t *doffs = nullptr, *dseeds = nullptr;
  int32_t *dfams = nullptr;
  int rc = 0;
  if (hipMalloc(&dp, sizeof(Piece) * (npieces ? npieces : 1)) != hipSuccess ||
      hipMalloc(&doffs, sizeof(uint64_t) * (count + 1)) != hipSuccess ||
      hipMalloc(&dseeds, sizeof(uint64_t) * count) != hipSuccess ||
      hipMalloc(&dfams, sizeof(int32_t) * count) != hipSuccess) {
    rc = -3;
  }
  if (rc == 0 &&
      (hipMemcpyAsync(dp, hp, sizeof(Piece) * npieces, hipMemcpyHostToDevice, s) != hipSuccess ||
       hipMemcpyAsync(doffs, h_offs, sizeof(uint64_t) * (count + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
       hipMemcpyAsync(dseeds, h_seeds, sizeof(uint64_t) * count, hipMemcpyHostToDevice, s) != hipSuccess ||
       hipMemcpyAsync(dfams, h_fams, sizeof(int32_t) * count, hipMemcpyHostToDevice, s) != hipSuccess)) {
    rc = -3;
  }
  if (rc == 0 && npieces) {
    hipLaunchKernelGGL(k_fill, dim3((uint32_t)npieces), dim3(256), 0, s, d_out, dt, dp, doffs, dfams, dseeds);
    hipLaunchKernelGGL(k_swaps, dim3((count + 63) / 64), dim3(64), 0, s, d_out, dt, doffs, dfams, dseeds, count);
    if (hipGetLastError() != hipSuccess) rc = -3;
  }
  if (hipStreamSynchronize(s) != hipSuccess) rc = -3;
  (void)hipFree(dp);
  (void)hipFree(doffs);
  (void)hipFree(dseeds);
  (void)hipFree(dfams);
  free(hp);
  return rc;
}

}  // extern "C"
