// The pass pair of Alg. 6 (X = A^T (A Q), or A (A^T Q) for Alg. 5) as one sweep over the rows
// of the forward product's segment matrix: for each row r, t_r = a_r Q is formed in registers
// from gathered rows of the short-side panel, and a_r^T t_r is added at once into the rows of
// X named by r's nonzeros with floating-point atomic adds, so the long-side panel Y = A Q is
// never stored or read back. The order of the adds into each row of X depends on timing: the
// result is not bitwise repeatable (it is exact whenever the sums are, e.g. on integer data).
//
// A wave owns a contiguous range of rows. Within a row the nonzeros are taken in pairs as in
// the paired-gather product: lanes 0-31 gather the even entry's panel row and lanes 32-63 the
// odd entry's, four columns per lane; the halves are added with a cross-half shuffle at the end
// of the row, after which both halves hold t_r, and the scatter takes the pairs again (lanes
// 0-31 the even entry's row of X, lanes 32-63 the odd one's).
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kFusedRowsPerWave = 16;

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

__global__ __launch_bounds__(256) void fused_pass_kernel(const int32_t* ptr, const int32_t* idx, const float* val,
                                                         int64_t nseg, const float* Q, int ldq, int lp, float* X,
                                                         int ldx) {
  const int lane = threadIdx.x & 63, half = lane >> 5;
  const int col = 4 * (lane & 31);
  const bool act = col < lp;
  const int gcol = act ? col : 0;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t r0 = w * kFusedRowsPerWave;
  const int64_t r1 = min(nseg, r0 + kFusedRowsPerWave);
  for (int64_t r = r0; r < r1; ++r) {
    const int p0 = ptr[r], p1 = ptr[r + 1];
    if (p0 == p1) continue;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int base = p0; base < p1; base += 64) {
      const int cnt = min(64, p1 - base);
      const int ci = lane < cnt ? idx[base + lane] : 0;
      const float vi = lane < cnt ? val[base + lane] : 0.f;
      for (int e = 0; e < cnt; e += 2) {
        const int src = e + half;
        // both shuffles run on every lane (a shuffle under a lane-dependent condition would read
        // lanes that the condition switched off); entries past the window weigh 0
        const int c = __shfl(ci, src & 63);
        const float vr = __shfl(vi, src & 63);
        const float v = src < cnt ? vr : 0.f;
        const float4 q = ld4(Q + (size_t)(src < cnt ? c : 0) * ldq + gcol);
        acc.x = fmaf(v, q.x, acc.x);
        acc.y = fmaf(v, q.y, acc.y);
        acc.z = fmaf(v, q.z, acc.z);
        acc.w = fmaf(v, q.w, acc.w);
      }
    }
    float4 t;
    t.x = acc.x + __shfl_xor(acc.x, 32);
    t.y = acc.y + __shfl_xor(acc.y, 32);
    t.z = acc.z + __shfl_xor(acc.z, 32);
    t.w = acc.w + __shfl_xor(acc.w, 32);
    for (int base = p0; base < p1; base += 64) {
      const int cnt = min(64, p1 - base);
      const int ci = lane < cnt ? idx[base + lane] : 0;
      const float vi = lane < cnt ? val[base + lane] : 0.f;
      for (int e = 0; e < cnt; e += 2) {
        const int src = e + half;
        const int c = __shfl(ci, src & 63);
        const float v = __shfl(vi, src & 63);
        if (src < cnt && act) {
          float* o = X + (size_t)c * ldx + col;
          unsafeAtomicAdd(o + 0, v * t.x);
          unsafeAtomicAdd(o + 1, v * t.y);
          unsafeAtomicAdd(o + 2, v * t.z);
          unsafeAtomicAdd(o + 3, v * t.w);
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void zero_panel_kernel(float* X, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) X[i] = 0.f;
}

}  // namespace

void launch_fused_pass(const int32_t* ptr, const int32_t* idx, const float* val, int64_t nseg, const float* Q,
                       int ldq, int lp, float* X, int ldx, int64_t xrows, hipStream_t st) {
  const int64_t count = xrows * (int64_t)ldx;
  if (count > 0) {
    const unsigned zg = (unsigned)std::min<int64_t>((count + 255) / 256, 65536);
    zero_panel_kernel<<<zg, 256, 0, st>>>(X, count);
  }
  if (nseg <= 0) return;
  const int64_t waves = (nseg + kFusedRowsPerWave - 1) / kFusedRowsPerWave;
  fused_pass_kernel<<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(ptr, idx, val, nseg, Q, ldq, lp, X, ldx);
}

}  // namespace frpca
