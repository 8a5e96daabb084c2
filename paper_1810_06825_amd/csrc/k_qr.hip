// Small FP64 kernels of the basic randomized PCA (Alg. 1 / Alg. 4, Sections 2.2 and 3.2):
// the orthonormalisation orth(X) by CholeskyQR2 and the SVD of the projected matrix B.
//
// orth(X): with G = X^T X (FP64 Gram of the FP32 panel, k_gram.hip), R = chol(G) upper
// triangular (G = R^T R) and Q = X R^-1 (k_tsmm.hip); repeated once on Q (CholeskyQR2), which
// leaves Q orthonormal to working precision whenever cond(X) stays well below 1e8. By Lemma 2
// any orthonormal basis of range(X) gives the algorithm the same result as the paper's
// Householder qr(X, 0).
//
// svd(B): B^T (a tall panel) = Q_B R with R the CholeskyQR2 factor R2 R1, and the SVD of the
// l x l factor R = U_R diag(sigma) W^T by one-sided (Hestenes) Jacobi applied to the columns of
// R^T: rotating them to mutual orthogonality gives R^T V = W diag(sigma), so the rotated
// columns, normalised, are the right singular vectors W of R (those of B^T, the left ones of
// B) and their norms the singular values; the rotations themselves are not kept. Results are
// handed over as sigma^2 ascending with W in the same column order, the layout of the
// eigendecomposition of the Gram matrix, so the final-step kernels of k_eig.hip apply as is.
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kQT = 1024;          // threads of the one-workgroup kernels
constexpr int kLd = kMaxL + 1;     // LDS row stride (odd: column walks spread over banks)

// Cholesky G = R^T R (R upper triangular, FP64) and its inverse, one workgroup.
// Rank guard: a pivot d_j <= tol * G_jj (the column's residual norm below sqrt(tol) of its
// own norm) or d_j <= 0 drops column j: row j of R is zero, column j of R^-1 is zero, so the
// column of Q = X R^-1 is zero and later columns ignore it. Outputs: Binv (l x ldb, zero
// padded, B[a*ldb + j] = (R^-1)[a][j]), R (l x l, ld l, optional), ndrop (optional).
__global__ __launch_bounds__(kQT) void chol_inv_kernel(const double* G, int ldg, int l, double tol, double* Binv,
                                                        int ldb, double* R, int* ndrop) {
  __shared__ double A[kMaxL * kLd];
  __shared__ double col[kMaxL];
  __shared__ double diag0[kMaxL];
  __shared__ int dropped[kMaxL];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < l * l; idx += kQT) {
    const int i = idx / l, k = idx - i * l;
    A[i * kLd + k] = (k >= i) ? G[(size_t)i * ldg + k] : 0.0;
  }
  for (int i = tid; i < l; i += kQT) diag0[i] = G[(size_t)i * ldg + i];
  __syncthreads();
  // right-looking factorization on the upper triangle
  for (int j = 0; j < l; ++j) {
    const double d = A[j * kLd + j];
    const bool drop = !(d > tol * diag0[j]) || !(d > 0.0);
    __syncthreads();
    if (drop) {
      for (int k = j + tid; k < l; k += kQT) A[j * kLd + k] = 0.0;
      if (tid == 0) dropped[j] = 1;
      __syncthreads();
      continue;
    }
    const double r = sqrt(d);
    const double rinv = 1.0 / r;
    for (int k = j + 1 + tid; k < l; k += kQT) A[j * kLd + k] *= rinv;
    if (tid == 0) {
      A[j * kLd + j] = r;
      dropped[j] = 0;
    }
    __syncthreads();
    // trailing update of the upper triangle: A[i][k] -= R[j][i] R[j][k], j < i <= k
    const int t = l - j - 1;
    for (int idx = tid; idx < t * t; idx += kQT) {
      const int i = j + 1 + idx / t, k = j + 1 + idx % t;
      if (k >= i) A[i * kLd + k] -= A[j * kLd + i] * A[j * kLd + k];
    }
    __syncthreads();
  }
  if (R)
    for (int idx = tid; idx < l * l; idx += kQT) {
      const int i = idx / l, k = idx - i * l;
      R[idx] = (k >= i) ? A[i * kLd + k] : 0.0;
    }
  if (ndrop && tid == 0) {
    int c = 0;
    for (int j = 0; j < l; ++j) c += dropped[j];
    *ndrop = c;
  }
  __syncthreads();
  // in-place inversion, column by column: with Z the inverse of the leading j x j block,
  // column j of R^-1 is -Z R[0:j, j] / R[j][j] over rows 0..j-1 and 1 / R[j][j] on the
  // diagonal. A dropped column j (zero row and diagonal) gets a zero column, and its zero row
  // keeps it out of every later column.
  for (int j = 0; j < l; ++j) {
    const bool drop = dropped[j] != 0;
    if (tid < j) col[tid] = A[tid * kLd + j];
    __syncthreads();
    if (!drop) {
      const double rjj_inv = 1.0 / A[j * kLd + j];
      if (tid < j) {
        double s = 0.0;
        for (int t = tid; t < j; ++t) s += A[tid * kLd + t] * col[t];
        A[tid * kLd + j] = -s * rjj_inv;
      }
      if (tid == 0) A[j * kLd + j] = rjj_inv;
    } else {
      if (tid <= j) A[tid * kLd + j] = 0.0;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < l * ldb; idx += kQT) {
    const int a = idx / ldb, j = idx - a * ldb;
    Binv[idx] = (j < l && j >= a) ? A[a * kLd + j] : 0.0;
  }
}

// C = A B for l x l FP64 matrices (ld l), one workgroup (R = R2 R1 of CholeskyQR2).
__global__ __launch_bounds__(kQT) void small_matmul_kernel(const double* Am, const double* Bm, int l, double* C) {
  for (int idx = threadIdx.x; idx < l * l; idx += kQT) {
    const int i = idx / l, j = idx - i * l;
    double s = 0.0;
    for (int t = 0; t < l; ++t) s += Am[(size_t)i * l + t] * Bm[(size_t)t * l + j];
    C[idx] = s;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One-sided Jacobi SVD of the l x l matrix R (ld l), applied to the columns of R^T (the rows
// of R) held in LDS as M[j][i] = R[j][i]. Round-robin pairing (circle method): in round r of
// a sweep, column L-1 meets column r and columns (r + i) and (r - i) (mod L-1) meet for
// i = 1 .. L/2-1, so a sweep of L-1 rounds meets every pair once with disjoint pairs inside
// a round; each wave rotates its pairs (a lane holds rows lane and lane+64 of both columns).
// A pair is rotated when |g| > tol sqrt(a b) (a, b, g the two squared norms and the inner
// product); sweeps stop after one without rotation (at most kMaxSweeps). Outputs: d = sigma^2
// ascending and W (l x l, row-major, column j the unit right singular vector of R paired with
// d[j]; zero for sigma = 0).
constexpr int kMaxSweeps = 40;
constexpr int kPW = (kMaxL / 2 + kQT / 64 - 1) / (kQT / 64);  // pairs per wave and round
__global__ __launch_bounds__(kQT) void jacobi_svd_kernel(const double* R, int l, double tol, double* d, double* W) {
  __shared__ double M[kMaxL * kLd];
  __shared__ double nrm2[kMaxL];
  __shared__ int any_rot;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kQT / 64;
  for (int idx = tid; idx < l * l; idx += kQT) {
    const int j = idx / l, i = idx - j * l;
    M[j * kLd + i] = R[idx];  // column j of R^T = row j of R
  }
  const int L = l + (l & 1);   // even player count (a dummy column when l is odd)
  const int npairs = L / 2;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    bool rotated = false;
    for (int r = 0; r < L - 1; ++r) {
      // a wave's pairs (at most kPW) are loaded and reduced together so their reductions overlap
      int pc[kPW], qc[kPW];
      bool ok[kPW];
      double x0[kPW], x1[kPW], y0[kPW], y1[kPW], sa[kPW], sb[kPW], sg[kPW];
#pragma unroll
      for (int u = 0; u < kPW; ++u) {
        const int pi = wave + u * nwaves;
        int p = 0, q = 0;
        if (pi == 0) {
          p = r;
          q = L - 1;
        } else {
          p = (r + pi) % (L - 1);
          q = (r - pi + (L - 1)) % (L - 1);
        }
        ok[u] = pi < npairs && p < l && q < l;  // q = L-1 = l is the dummy column of odd l
        pc[u] = ok[u] ? p : 0;
        qc[u] = ok[u] ? q : 0;
        x0[u] = (ok[u] && lane < l) ? M[pc[u] * kLd + lane] : 0.0;
        x1[u] = (ok[u] && lane + 64 < l) ? M[pc[u] * kLd + lane + 64] : 0.0;
        y0[u] = (ok[u] && lane < l) ? M[qc[u] * kLd + lane] : 0.0;
        y1[u] = (ok[u] && lane + 64 < l) ? M[qc[u] * kLd + lane + 64] : 0.0;
        sa[u] = x0[u] * x0[u] + x1[u] * x1[u];
        sb[u] = y0[u] * y0[u] + y1[u] * y1[u];
        sg[u] = x0[u] * y0[u] + x1[u] * y1[u];
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int u = 0; u < kPW; ++u) {
          sa[u] += __shfl_xor(sa[u], off);
          sb[u] += __shfl_xor(sb[u], off);
          sg[u] += __shfl_xor(sg[u], off);
        }
      }
#pragma unroll
      for (int u = 0; u < kPW; ++u) {
        const double a = sa[u], b = sb[u], g = sg[u];
        if (ok[u] && g != 0.0 && fabs(g) > tol * sqrt(a * b)) {
          rotated = true;
          const double zeta = (b - a) / (2.0 * g);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double sn = c * t;
          if (lane < l) {
            M[pc[u] * kLd + lane] = c * x0[u] - sn * y0[u];
            M[qc[u] * kLd + lane] = sn * x0[u] + c * y0[u];
          }
          if (lane + 64 < l) {
            M[pc[u] * kLd + lane + 64] = c * x1[u] - sn * y1[u];
            M[qc[u] * kLd + lane + 64] = sn * x1[u] + c * y1[u];
          }
        }
      }
      __syncthreads();
    }
    if (rotated && lane == 0) any_rot = 1;
    __syncthreads();
    const int go = any_rot;
    __syncthreads();
    if (!go) break;
  }
  // column norms, then ranks for the ascending order (ties by index)
  for (int j = wave; j < l; j += nwaves) {
    const double v0 = lane < l ? M[j * kLd + lane] : 0.0, v1 = lane + 64 < l ? M[j * kLd + lane + 64] : 0.0;
    const double s = wave_sum(v0 * v0 + v1 * v1);
    if (lane == 0) nrm2[j] = s;
  }
  __syncthreads();
  for (int j = wave; j < l; j += nwaves) {
    const double sj = nrm2[j];
    int rank = 0;
    for (int t = 0; t < l; ++t) {
      const double st = nrm2[t];
      rank += (st < sj || (st == sj && t < j)) ? 1 : 0;
    }
    const double inv = sj > 0.0 ? 1.0 / sqrt(sj) : 0.0;
    for (int i = lane; i < l; i += 64) W[(size_t)i * l + rank] = M[j * kLd + i] * inv;
    if (lane == 0) d[rank] = sj;
  }
}

}  // namespace

void launch_chol_inv(const double* G, int ldg, int l, double tol, double* Binv, int ldb, double* R, int* ndrop,
                     hipStream_t st) {
  chol_inv_kernel<<<1, kQT, 0, st>>>(G, ldg, l, tol, Binv, ldb, R, ndrop);
}

void launch_small_matmul(const double* A, const double* B, int l, double* C, hipStream_t st) {
  small_matmul_kernel<<<1, kQT, 0, st>>>(A, B, l, C);
}

void launch_jacobi_svd(const double* R, int l, double tol, double* d, double* W, hipStream_t st) {
  jacobi_svd_kernel<<<1, kQT, 0, st>>>(R, l, tol, d, W);
}

}  // namespace frpca
