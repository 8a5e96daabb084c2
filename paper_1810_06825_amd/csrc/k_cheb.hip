// Panel kernels of eigSVDs (Alg. 3) on the GPU: the three-term recurrence of the Chebyshev
// filter that accelerates the subspace iteration on B = A^T A, and the Ritz residual norms
// that decide convergence.
#include "kernels.h"

namespace frpca {
namespace {

// out = a * X + b * Y + c * Z over rows x cols (leading dimension ld); Z may be null (c = 0)
// and out may alias Z (each element is read before it is written, by the same thread).
__global__ __launch_bounds__(256) void panel_comb_kernel(int64_t rows, int cols, int ld, float a, const float* X,
                                                         float b, const float* Y, float c, const float* Z,
                                                         float* out) {
  const int64_t total = rows * (int64_t)ld;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int j = (int)(i % ld);
    float v = 0.f;
    if (j < cols) {
      v = a * X[i] + b * Y[i];
      if (Z) v += c * Z[i];
    }
    out[i] = v;
  }
}

// Partial sums over blocks of rows of (Z[r][j] - theta_j Q[r][j])^2, in FP64, for j < l:
// part[block][j].
constexpr int kResRows = 2048;
__global__ __launch_bounds__(256) void resid_partial_kernel(const float* Q, const float* Z, int ld, int64_t rows,
                                                            int l, const double* theta, double* part) {
  __shared__ double red[4][kMaxL];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int64_t r0 = (int64_t)blockIdx.x * kResRows, r1 = min(rows, r0 + kResRows);
  // lane covers columns lane and lane + 64; the four waves take every fourth row
  double s0 = 0.0, s1 = 0.0;
  const double th0 = lane < l ? theta[lane] : 0.0, th1 = lane + 64 < l ? theta[lane + 64] : 0.0;
  for (int64_t r = r0 + wave; r < r1; r += 4) {
    if (lane < l) {
      const double d = (double)Z[r * ld + lane] - th0 * (double)Q[r * ld + lane];
      s0 += d * d;
    }
    if (lane + 64 < l) {
      const double d = (double)Z[r * ld + lane + 64] - th1 * (double)Q[r * ld + lane + 64];
      s1 += d * d;
    }
  }
  red[wave][lane] = s0;
  red[wave][lane + 64] = s1;
  __syncthreads();
  if (t < l) part[(size_t)blockIdx.x * kMaxL + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

// out[j] = sum over blocks (in block order) of part[block][j].
__global__ __launch_bounds__(kMaxL) void resid_final_kernel(const double* part, int64_t nblk, int l, double* out) {
  const int j = threadIdx.x;
  if (j >= l) return;
  double s = 0.0;
  for (int64_t b = 0; b < nblk; ++b) s += part[(size_t)b * kMaxL + j];
  out[j] = s;
}

// G = (G + G^T) / 2 in place (l x l, ld l): the Rayleigh quotient Q^T (B Q) of a symmetric B
// is symmetric up to rounding, and the eigensolver reads the whole matrix.
__global__ __launch_bounds__(1024) void symmetrize_kernel(double* G, int l) {
  for (int idx = threadIdx.x; idx < l * l; idx += 1024) {
    const int i = idx / l, j = idx - i * l;
    if (j > i) {
      const double v = 0.5 * (G[(size_t)i * l + j] + G[(size_t)j * l + i]);
      G[(size_t)i * l + j] = v;
      G[(size_t)j * l + i] = v;
    }
  }
}

}  // namespace

void launch_symmetrize(double* G, int l, hipStream_t st) { symmetrize_kernel<<<1, 1024, 0, st>>>(G, l); }

void launch_panel_comb(int64_t rows, int cols, int ld, float a, const float* X, float b, const float* Y, float c,
                       const float* Z, float* out, hipStream_t st) {
  const int64_t total = rows * (int64_t)ld;
  if (total <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  panel_comb_kernel<<<grid, 256, 0, st>>>(rows, cols, ld, a, X, b, Y, c, Z, out);
}

size_t resid_temp_bytes(int64_t rows) {
  return (size_t)((rows + kResRows - 1) / kResRows + 1) * kMaxL * sizeof(double);
}

void launch_resid_norms(const float* Q, const float* Z, int ld, int64_t rows, int l, const double* theta,
                        double* temp, double* out, hipStream_t st) {
  const int64_t nblk = std::max<int64_t>(1, (rows + kResRows - 1) / kResRows);
  resid_partial_kernel<<<(unsigned)nblk, 256, 0, st>>>(Q, Z, ld, rows, l, theta, temp);
  resid_final_kernel<<<1, kMaxL, 0, st>>>(temp, nblk, l, out);
}

}  // namespace frpca
