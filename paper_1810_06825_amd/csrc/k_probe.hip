// Ceiling of the sparse products' access pattern: random 512-byte row gathers in the products'
// lane shape (lanes 0-31 read one row of 128 floats as float4, lanes 32-63 another, eight row
// pairs in flight per wave), with no arithmetic beyond a running sum. What it sustains is the
// rate the gathers of A Q and A^T Y can reach on the machine, beside the streaming peak.
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kProbeBatch = 8;  // row pairs in flight per wave

__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(256) void gather_probe_kernel(const float* P, int64_t rows, int ld, int pairs_per_wave,
                                                           uint32_t seed, float sentinel, float* out) {
  const int lane = threadIdx.x & 63, half = lane >> 5, l32 = lane & 31;
  const uint32_t w = blockIdx.x * 4u + (threadIdx.x >> 6);
  float acc = 0.f;
  for (int it = 0; it < pairs_per_wave; it += kProbeBatch) {
    float4 v[kProbeBatch];
#pragma unroll
    for (int u = 0; u < kProbeBatch; ++u) {
      const uint32_t h = probe_hash(seed ^ probe_hash(w * 0x9e3779b9u + 2u * (uint32_t)(it + u) + (uint32_t)half));
      const int64_t r = (int64_t)(h % (uint32_t)rows);
      v[u] = *reinterpret_cast<const float4*>(P + (size_t)r * ld + 4 * l32);
    }
#pragma unroll
    for (int u = 0; u < kProbeBatch; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  if (acc == sentinel) out[lane] = acc;  // keeps the loads; the host passes a value no sum takes
}

}  // namespace

// rows read per workgroup: four waves, each 32 batches of 8 row pairs
constexpr int64_t kProbeRowsPerBlock = 4 * 2 * (int64_t)kProbeBatch * 32;

int64_t gather_probe_rows(int64_t gathers) {
  const int64_t blocks = std::max<int64_t>(1, (gathers + kProbeRowsPerBlock - 1) / kProbeRowsPerBlock);
  return blocks * kProbeRowsPerBlock;
}

void launch_gather_probe(const float* P, int64_t rows, int ld, int64_t gathers, uint32_t seed, float* out,
                         hipStream_t st) {
  const int64_t blocks = gather_probe_rows(gathers) / kProbeRowsPerBlock;
  gather_probe_kernel<<<(unsigned)blocks, 256, 0, st>>>(P, rows, ld, kProbeBatch * 32, seed, -1.0e38f, out);
}

}  // namespace frpca
