// Gaussian test matrix of Alg. 5/6 ("randn"): Philox4x32-10 words turned into normals by
// the Box-Muller transform in FP64, rounded to FP32.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds on a 4x32-bit counter with
// a 2x32-bit key; each round multiplies counter words 0 and 2 by 0xD2511F53 and
// 0xCD9E8D57 (64-bit products), mixes the high halves with words 1 and 3 and the key, and
// the key is bumped by 0x9E3779B9 / 0xBB67AE85 between rounds. Normal number t of the
// stream with key `seed` comes from block b = t/4 (counter = (b lo, b hi, 0, 0)); words
// (x0, x1) give normals 4b, 4b+1 and (x2, x3) give 4b+2, 4b+3 via
// u1 = (x+1) 2^-32, u2 = x 2^-32, z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).
#include "kernels.h"

namespace frpca {
namespace {

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

__device__ __forceinline__ void put(float* f32, uint16_t* b16, int64_t r, int j, int ld, float v) {
  const size_t o = (size_t)r * ld + j;
  if (f32) f32[o] = v;
  if (b16) b16[o] = f32_to_bf16(v);
}

// One thread per Philox block: writes normals 4b..4b+3 and, for any row whose last
// element it writes, that row's pad columns.
__global__ __launch_bounds__(256) void gaussian_kernel(uint64_t seed, int64_t rows, int l, int ld,
                                                       float* f32, uint16_t* b16) {
  const int64_t total = rows * (int64_t)l;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b * 4 >= total) return;
  uint32_t c0 = (uint32_t)b, c1 = (uint32_t)((uint64_t)b >> 32), c2 = 0, c3 = 0;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double two32 = 2.3283064365386963e-10;  // 2^-32
  const double twopi = 6.283185307179586;
  double z[4];
  {
    const double u1 = ((double)c0 + 1.0) * two32, u2 = (double)c1 * two32;
    const double rad = sqrt(-2.0 * log(u1));
    z[0] = rad * cos(twopi * u2);
    z[1] = rad * sin(twopi * u2);
  }
  {
    const double u1 = ((double)c2 + 1.0) * two32, u2 = (double)c3 * two32;
    const double rad = sqrt(-2.0 * log(u1));
    z[2] = rad * cos(twopi * u2);
    z[3] = rad * sin(twopi * u2);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t t = b * 4 + i;
    if (t >= total) break;
    const int64_t r = t / l;
    const int j = (int)(t - r * l);
    put(f32, b16, r, j, ld, (float)z[i]);
    if (j == l - 1)
      for (int p = l; p < ld; ++p) put(f32, b16, r, p, ld, 0.0f);
  }
}

}  // namespace

void launch_gaussian(uint64_t seed, int64_t rows, int l, int ld, float* out_f32,
                     uint16_t* out_bf16, hipStream_t st) {
  const int64_t total = rows * (int64_t)l;
  if (total <= 0) return;
  const int64_t blocks = (total + 3) / 4;
  const int64_t grid = (blocks + 255) / 256;
  gaussian_kernel<<<dim3((unsigned)grid), dim3(256), 0, st>>>(seed, rows, l, ld, out_f32, out_bf16);
}

}  // namespace frpca
