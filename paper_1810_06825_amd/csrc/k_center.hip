// Principal components of the column-centred matrix A - 1 mu^T (mu = column means) without
// forming it: the paper's PCA assumes centred data (Section 1), which a sparse matrix cannot
// store. Each product of the method becomes a sparse product plus a rank-1 term,
//   (A - 1 mu^T) X   = A X   - 1 (mu^T X)      (every output row minus the row vector mu^T X)
//   (A - 1 mu^T)^T Y = A^T Y - mu (1^T Y)      (output row j minus mu_j times the column sums of Y)
// and the rank-1 terms are applied where the products write their output rows. This file
// holds the column means, the weighted column sums of a panel (mu^T X and 1^T Y) and the
// per-column term of the centred backward.
#include "kernels.h"

namespace frpca {
namespace {

// One wave per column: FP64 partial sums per lane, then a fixed xor-butterfly, so the result
// does not depend on timing.
__global__ __launch_bounds__(256) void colmean_kernel(const int32_t* cp, const float* val, int64_t n, int64_t m,
                                                      float* mu) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int64_t e = cp[c] + lane; e < cp[c + 1]; e += 64) s += (double)val[e];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) mu[c] = (float)(s / (double)m);
}

constexpr int kWsumBlocks = 512;  // blocks of the weighted column sums (each a stretch of rows)

// Block partials of sum_r w[r] P[r, :] (w = 1 when null) in FP64. A half-wave takes one row
// (lane L covers columns 4 (L mod 32) .. + 3), so a block of 4 waves walks 8 rows at a time
// through its stretch; the 8 row streams are added in a fixed order through LDS.
template <bool BF16>
__global__ __launch_bounds__(256) void wsum_partial_kernel(const void* P, int ldp, int64_t rows, int lp, const float* w,
                                                           double* part) {
  __shared__ double sh[8][128];
  const int t = threadIdx.x, stream = t >> 5, c0 = 4 * (t & 31);
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = min(rows, r0 + per);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int64_t r = r0 + stream; r < r1; r += 8) {
    const double wr = w ? (double)w[r] : 1.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (c0 + q < lp) {
        const size_t o = (size_t)r * ldp + c0 + q;
        const double x = BF16 ? (double)bf16_to_f32(static_cast<const uint16_t*>(P)[o])
                              : (double)static_cast<const float*>(P)[o];
        s[q] += wr * x;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) sh[stream][c0 + q] = s[q];
  __syncthreads();
  if (t < 128) {
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) tot += sh[i][t];
    part[(size_t)blockIdx.x * 128 + t] = tot;
  }
}

// v[c] = scale * (sum of the block partials in block order)
__global__ __launch_bounds__(128) void wsum_final_kernel(const double* part, int64_t nblk, int lp, double scale,
                                                         float* v) {
  const int c = threadIdx.x;
  if (c >= lp) return;
  double s = 0.0;
#pragma unroll 8
  for (int64_t b = 0; b < nblk; ++b) s += part[(size_t)b * 128 + c];
  v[c] = (float)(scale * s);
}

// corr[c] = a . V[c, :] + b . R[c, :] (k-vectors a, b; R may be null; V and R with leading
// dimension ld)
__global__ __launch_bounds__(256) void center_corr_kernel(const float* a, const float* V, const float* b,
                                                          const float* R, int64_t n, int k, int ld, float* corr) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  double s = 0.0;
  for (int i = 0; i < k; ++i) {
    s += (double)a[i] * (double)V[(size_t)c * ld + i];
    if (R) s += (double)b[i] * (double)R[(size_t)c * ld + i];
  }
  corr[c] = (float)s;
}

// dst[r, c] = src[r, c] for c < cols, 0 for cols <= c < ldd (one thread per destination entry)
__global__ __launch_bounds__(256) void pad_copy_kernel(const float* src, int lds, int64_t rows, int cols, float* dst,
                                                       int ldd) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * ldd) return;
  const int64_t r = idx / ldd;
  const int c = (int)(idx - r * ldd);
  dst[idx] = c < cols ? src[(size_t)r * lds + c] : 0.f;
}

}  // namespace

void launch_pad_copy(const float* src, int lds, int64_t rows, int cols, float* dst, int ldd, hipStream_t st) {
  const int64_t total = rows * ldd;
  if (total <= 0) return;
  pad_copy_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(src, lds, rows, cols, dst, ldd);
}

void launch_colmean(const int32_t* cp, const float* val, int64_t n, int64_t m, float* mu, hipStream_t st) {
  if (n <= 0) return;
  colmean_kernel<<<(unsigned)((n + 3) / 4), 256, 0, st>>>(cp, val, n, m, mu);
}

size_t wsum_temp_bytes(int64_t rows) {
  (void)rows;
  return (size_t)kWsumBlocks * 128 * sizeof(double);
}

void launch_wsum(const void* P, bool bf16, int ldp, int64_t rows, int lp, const float* w, double scale, double* part,
                 float* v, hipStream_t st) {
  const int64_t nblk = rows < kWsumBlocks ? (rows > 0 ? rows : 0) : kWsumBlocks;
  if (nblk > 0) {
    if (bf16) wsum_partial_kernel<true><<<(unsigned)nblk, 256, 0, st>>>(P, ldp, rows, lp, w, part);
    else wsum_partial_kernel<false><<<(unsigned)nblk, 256, 0, st>>>(P, ldp, rows, lp, w, part);
  }
  wsum_final_kernel<<<1, 128, 0, st>>>(part, nblk, lp, scale, v);
}

void launch_center_corr(const float* a, const float* V, const float* b, const float* R, int64_t n, int k, int ld,
                        float* corr, hipStream_t st) {
  if (n <= 0) return;
  center_corr_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a, V, b, R, n, k, ld, corr);
}

}  // namespace frpca
