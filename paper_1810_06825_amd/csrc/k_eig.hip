// Small epilogues of eigSVD (Alg. 2 steps 3-5) and of the final steps of Alg. 5/6: basis
// coefficients from the eigenpairs of the Gram matrix, the final selection, and the sign
// convention. The eigendecomposition itself (Alg. 2 step 2) is in k_syev.hip.
#include "kernels.h"

namespace frpca {
namespace {

// eigSVD basis coefficients (Alg. 2 steps 3-5): B = W diag(1/sigma), sigma = sqrt(max(d,0)),
// columns with sigma <= tol * max(sigma) zeroed. B is l x l with leading dimension ldb.
__global__ __launch_bounds__(256) void eigsvd_coeffs_kernel(const double* d, const double* W, int l, int ldb,
                                                            double tol, double* B, double* sigma) {
  const double smax = sqrt(fmax(d[l - 1], 0.0));
  for (int idx = threadIdx.x + blockIdx.x * blockDim.x; idx < l * ldb; idx += blockDim.x * gridDim.x) {
    const int a = idx / ldb, j = idx - a * ldb;
    double v = 0.0;
    if (j < l) {
      const double s = sqrt(fmax(d[j], 0.0));
      if (s > tol * smax && s > 0.0) v = W[(size_t)a * l + j] / s;
    }
    B[idx] = v;
  }
  if (sigma && blockIdx.x == 0)
    for (int j = threadIdx.x; j < l; j += blockDim.x) {
      const double s = sqrt(fmax(d[j], 0.0));
      sigma[j] = (s > tol * smax && s > 0.0) ? s : 0.0;
    }
}

// Final selection ind = l-1, ..., l-k (k+s:-1:s+1 in the paper's 1-based notation).
__global__ __launch_bounds__(256) void final_coeffs_kernel(const double* d, const double* W, int l, int k, int ldb,
                                                           double rank_tol, double* Blong, double* Bshort,
                                                           float* S, float* S_keep, int* ndropped) {
  const double smax = sqrt(fmax(d[l - 1], 0.0));
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < l * ldb) {
    const int a = idx / ldb, i = idx - a * ldb;
    double bl = 0.0, bs = 0.0;
    if (i < k) {
      const int j = l - 1 - i;
      const double s = sqrt(fmax(d[j], 0.0));
      if (s > rank_tol * smax && s > 0.0) {
        bs = W[(size_t)a * l + j];
        bl = bs / s;
      }
    }
    Blong[idx] = bl;
    Bshort[idx] = bs;
  }
  if (blockIdx.x == 0) {
    // S and the number of dropped values (k <= 128 < blockDim): per-wave ballot counts
    __shared__ int nd_w[4];
    const int i = threadIdx.x;
    bool drop = false;
    if (i < k) {
      const double s = sqrt(fmax(d[l - 1 - i], 0.0));
      const bool keep = s > rank_tol * smax && s > 0.0;
      S[i] = keep ? (float)s : 0.0f;
      if (S_keep) S_keep[i] = S[i];
      drop = !keep;
    }
    const uint64_t m = __ballot(drop);
    if ((i & 63) == 0) nd_w[i >> 6] = (int)__popcll(m);
    __syncthreads();
    if (i == 0) *ndropped = nd_w[0] + nd_w[1] + nd_w[2] + nd_w[3];
  }
}

// Sign convention: per column i of V (rows x k, ld k), the largest |entry| (ties: lowest
// row). Pass 1: one partial (|v|, row) per block and column; pass 2 reduces in block order.
constexpr int kSignRows = 32;

__global__ __launch_bounds__(256) void sign_partial_kernel(const float* V, int64_t rows, int k, float* pv, int* pr) {
  const int64_t r0 = (int64_t)blockIdx.x * kSignRows;
  const int64_t r1 = min(rows, r0 + kSignRows);
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    float best = -1.0f;
    int brow = 0;
#pragma unroll 8
    for (int64_t r = r0; r < r1; ++r) {
      const float a = fabsf(V[r * k + i]);
      if (a > best) {
        best = a;
        brow = (int)r;
      }
    }
    pv[(size_t)blockIdx.x * k + i] = best;
    pr[(size_t)blockIdx.x * k + i] = brow;
  }
}

// One block per column i: reduce the per-block candidates (|v|, row) in block order (ties:
// lowest row), then fold the sign into column i of both coefficient matrices (B_other may be
// null), so either factor rebuilt from them carries the convention.
__global__ __launch_bounds__(256) void sign_final_kernel(const float* V, int k, int nblk, const float* pv,
                                                         const int* pr, float* sgn, double* Blong, double* B_other,
                                                         int ldb, int l) {
  __shared__ float sv[256];
  __shared__ int sr[256];
  const int i = blockIdx.x, t = threadIdx.x;
  float best = -1.0f;
  int brow = 0;
  for (int b = t; b < nblk; b += 256) {
    const float a = pv[(size_t)b * k + i];
    const int r = pr[(size_t)b * k + i];
    if (a > best || (a == best && r < brow)) {
      best = a;
      brow = r;
    }
  }
  sv[t] = best;
  sr[t] = brow;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      const float a = sv[t + off];
      const int r = sr[t + off];
      if (a > sv[t] || (a == sv[t] && r < sr[t])) {
        sv[t] = a;
        sr[t] = r;
      }
    }
    __syncthreads();
  }
  const float s = (V[(size_t)sr[0] * k + i] < 0.0f) ? -1.0f : 1.0f;
  if (t == 0) sgn[i] = s;
  if (s < 0.0f)
    for (int a = t; a < l; a += 256) {
      Blong[(size_t)a * ldb + i] = -Blong[(size_t)a * ldb + i];
      if (B_other) B_other[(size_t)a * ldb + i] = -B_other[(size_t)a * ldb + i];
    }
}

__global__ __launch_bounds__(256) void sign_apply_kernel(float* V, int64_t rows, int k, const float* sgn) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * k) return;
  const int i = (int)(idx % k);
  if (sgn[i] < 0.0f) V[idx] = -V[idx];
}

}  // namespace

void launch_eigsvd_coeffs(const double* d, const double* W, int l, int ldb, double tol, double* B, double* sigma,
                          hipStream_t st) {
  const int total = l * ldb;
  eigsvd_coeffs_kernel<<<(total + 255) / 256, 256, 0, st>>>(d, W, l, ldb, tol, B, sigma);
}

void launch_final_coeffs(const double* d, const double* W, int l, int k, int ldb, double rank_tol, double* Blong,
                         double* Bshort, float* S, float* S_keep, int* ndropped, hipStream_t st) {
  final_coeffs_kernel<<<(l * ldb + 255) / 256, 256, 0, st>>>(d, W, l, k, ldb, rank_tol, Blong, Bshort, S, S_keep,
                                                            ndropped);
}

size_t sign_partial_bytes(int64_t rows, int k) {
  const int64_t nblk = (rows + kSignRows - 1) / kSignRows;
  return (size_t)nblk * k * (sizeof(float) + sizeof(int)) + (size_t)k * sizeof(float) + 256;
}

void launch_sign_fix(float* V, int64_t rows, int k, double* Blong, double* B_other, int ldb, int brows, void* partial,
                     hipStream_t st) {
  const int64_t nblk = (rows + kSignRows - 1) / kSignRows;
  float* pv = static_cast<float*>(partial);
  int* pr = reinterpret_cast<int*>(pv + nblk * k);
  float* sgn = reinterpret_cast<float*>(pr + nblk * k);
  sign_partial_kernel<<<(unsigned)nblk, 256, 0, st>>>(V, rows, k, pv, pr);
  sign_final_kernel<<<k, 256, 0, st>>>(V, k, (int)nblk, pv, pr, sgn, Blong, B_other, ldb, brows);
  sign_apply_kernel<<<(unsigned)((rows * k + 255) / 256), 256, 0, st>>>(V, rows, k, sgn);
}

}  // namespace frpca
