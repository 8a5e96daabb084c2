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

// A lane's double from another lane of its row of 16, by a DPP control (two 32-bit moves).
template <int kCtrl>
__device__ __forceinline__ double dpp_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// 1 / x and 1 / sqrt(x) for x > 0 from the hardware estimates, each refined by two
// Newton-Raphson steps (the error squares with each step; two take the estimate to the
// rounding level). Much shorter dependency chains than the IEEE-rounded division and square
// root, which these kernels' per-step latency is made of.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-h * y, y, 0.5);  // y (3 - x y^2) / 2 = y + y (1/2 - (x/2) y^2)
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

// Sum over each aligned group of eight lanes (every lane of the group gets the sum): swaps
// within pairs and within quads (quad_perm [1,0,3,2] and [2,3,0,1]), then the mirror of the
// group (lane i with lane 7 - i, row_half_mirror), which pairs each quad with the other.
// All eight lanes of a group must be active.
__device__ __forceinline__ double sum8(double v) {
  v += dpp_double<0xB1>(v);
  v += dpp_double<0x4E>(v);
  v += dpp_double<0x141>(v);
  return v;
}

// Cholesky G = R^T R (R upper triangular, FP64) and its inverse, one workgroup.
// Rank guard: a pivot d_j <= tol * G_jj (the column's residual norm below sqrt(tol) of its
// own norm) or d_j <= 0 drops column j: row j of R is zero, column j of R^-1 is zero, so the
// column of Q = X R^-1 is zero and later columns ignore it. Outputs: Binv (l x ldb, zero
// padded, B[a*ldb + j] = (R^-1)[a][j]), R (l x l, ld l, optional), ndrop (optional).
//
// Both halves take one barrier per column and issue LDS work only for the live part of the
// triangle (the kernel is bound by LDS accesses and barrier latency, not arithmetic).
// Factorization, step j: the trailing update A[i][k] -= A[j][i] A[j][k] / d_j (j < i <= k)
// with row j unscaled (rows are scaled by 1 / sqrt(d_j) after the last step); a wave owns
// rows i (every 16th), its lanes the columns j + 1 + lane and j + 65 + lane, and the loads of
// four rows are issued before their stores. Inversion, step j:
// column j of R^-1 is -Z R[0:j, j] / R[j][j] with Z the inverse of the leading j x j block
// (already in place); R[0:j+1, j] was copied to LDS during step j - 1 (double buffer), eight
// lanes share a row's dot product, four terms in flight per lane.
constexpr int kCholSub = 8;     // lanes per row in the inversion's dot products
constexpr int kCholWaves = kQT / 64;
constexpr int kRowBatch = 4;    // rows whose loads are in flight together (trailing update)
__global__ __launch_bounds__(kQT) void chol_inv_kernel(const double* G, int ldg, int l, double tol, double* Binv,
                                                        int ldb, double* R, int* ndrop) {
  __shared__ double A[kMaxL * kLd];
  __shared__ double colbuf[2][kMaxL];
  __shared__ double diag0[kMaxL];
  __shared__ double dinv_all[kMaxL];
  __shared__ double piv[kMaxL];
  __shared__ int dropped[kMaxL];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < l * l; idx += kQT) {
    const int i = idx / l, k = idx - i * l;
    A[i * kLd + k] = (k >= i) ? G[(size_t)i * ldg + k] : 0.0;
  }
  for (int i = tid; i < l; i += kQT) diag0[i] = G[(size_t)i * ldg + i];
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    const double d = A[j * kLd + j];
    const bool drop = !(d > tol * diag0[j]) || !(d > 0.0);
    if (tid == 0) {
      dropped[j] = drop ? 1 : 0;
      piv[j] = d;
    }
    if (!drop) {
      const int k0 = j + 1 + lane, k1 = k0 + 64;
      const bool two = j + 65 < l;  // wave-uniform: a second column slot is live
      const double r0 = k0 < l ? A[j * kLd + k0] : 0.0;
      const double r1 = (two && k1 < l) ? A[j * kLd + k1] : 0.0;
      const double dinv = rcp_nr(d);
      for (int ib = j + 1 + wave; ib < l; ib += kCholWaves * kRowBatch) {
        double f[kRowBatch], v0[kRowBatch], v1[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          const int i = ib + u * kCholWaves;
          const bool live = i < l;  // wave-uniform
          f[u] = live ? A[j * kLd + i] : 0.0;
          v0[u] = (live && k0 < l && k0 >= i) ? A[i * kLd + k0] : 0.0;
          v1[u] = (live && two && k1 < l && k1 >= i) ? A[i * kLd + k1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          const int i = ib + u * kCholWaves;
          const double fu = f[u] * dinv;
          if (i < l && k0 < l && k0 >= i) A[i * kLd + k0] = v0[u] - fu * r0;
          if (i < l && two && k1 < l && k1 >= i) A[i * kLd + k1] = v1[u] - fu * r1;
        }
      }
    }
    __syncthreads();
  }
  // rows of R: row j of the reduced matrix over sqrt(d_j) (zero for a dropped column)
  for (int idx = tid; idx < l * l; idx += kQT) {
    const int i = idx / l, k = idx - i * l;
    if (k < i) continue;
    const double di = piv[i];
    const double v = dropped[i] ? 0.0 : (k == i ? sqrt(di) : A[i * kLd + k] / sqrt(di));
    A[i * kLd + k] = v;
  }
  __syncthreads();
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
  // in-place inversion, column by column. A dropped column j (zero row and diagonal) gets a
  // zero column, and its zero row keeps it out of every later column. colbuf[j & 1][0..j]
  // holds column j of R down to the diagonal; the reciprocals of the diagonal are taken first.
  for (int j = tid; j < l; j += kQT) dinv_all[j] = dropped[j] ? 0.0 : 1.0 / A[j * kLd + j];
  if (tid == 0 && l > 0) colbuf[0][0] = A[0];
  __syncthreads();
  const int row = tid / kCholSub, sub = tid % kCholSub;
  for (int j = 0; j < l; ++j) {
    // prefetch R[0:j+1, j+1] for the next step (column j+1 is untouched until then): loaded
    // here, stored after the dot products
    const bool pf = j + 1 < l && tid <= j + 1;
    const double pv = pf ? A[tid * kLd + j + 1] : 0.0;
    const double* cb = colbuf[j & 1];
    const double rjj_inv = dinv_all[j];
    if (row < j) {
      double s = 0.0;
      for (int t0 = row + sub; t0 < j; t0 += 4 * kCholSub) {
        double av[4], cv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = t0 + u * kCholSub;
          av[u] = t < j ? A[row * kLd + t] : 0.0;
          cv[u] = t < j ? cb[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s += av[u] * cv[u];
      }
      s = sum8(s);
      if (sub == 0) A[row * kLd + j] = -s * rjj_inv;
    }
    if (tid == 0) A[j * kLd + j] = rjj_inv;
    if (pf) colbuf[(j + 1) & 1][tid] = pv;
    __syncthreads();
  }
  for (int idx = tid; idx < l * ldb; idx += kQT) {
    const int a = idx / ldb, j = idx - a * ldb;
    Binv[idx] = (j < l && j >= a) ? A[a * kLd + j] : 0.0;
  }
}

// C = A B for l x l FP64 matrices (ld l) (R = R2 R1 of CholeskyQR2): workgroup i forms row i,
// thread j its entry j (the reads of B run along rows).
__global__ __launch_bounds__(kMaxL) void small_matmul_kernel(const double* Am, const double* Bm, int l, double* C) {
  __shared__ double arow[kMaxL];
  const int i = blockIdx.x, j = threadIdx.x;
  if (j < l) arow[j] = Am[(size_t)i * l + j];
  __syncthreads();
  if (j >= l) return;
  double s = 0.0;
  for (int t = 0; t < l; ++t) s += arow[t] * Bm[(size_t)t * l + j];
  C[(size_t)i * l + j] = s;
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
// a round. Eight lanes hold a pair (rows sub, sub + 8, ... of both columns, in registers for
// the round), so a wave works on eight pairs at once and the rotation of each is computed
// once per lane group; one barrier per round. A pair is rotated when |g| > tol sqrt(a b)
// (a, b, g the two squared norms and the inner product); sweeps stop after one without
// rotation (at most kMaxSweeps). Outputs: d = sigma^2 ascending and W (l x l, row-major,
// column j the unit right singular vector of R paired with d[j]; zero for sigma = 0).
constexpr int kMaxSweeps = 40;
constexpr int kJT = 512;                    // most threads: kJSub lanes for each of up to kMaxL / 2 pairs
constexpr int kJSub = 8;                    // lanes per pair (the groups of sum8)
// LDS column stride: 136 doubles puts consecutive columns 16 banks apart, so the eight lane
// groups of a wave (consecutive columns, 16 words each) spread over the banks
constexpr int kLdJ = kMaxL + 8;
static_assert(kJT == kMaxL / 2 * kJSub, "one lane group per pair");
// kRows rows of a column per lane (8 kRows >= l). The columns are stored padded with zero rows
// up to 8 kRows, and a zero dummy column joins them when l is odd, so a round runs without
// bounds tests: the padding stays zero under rotations, and a pair with a zero column has
// g = 0 and is never rotated. Launched with one lane group per pair (blockDim.x = 8 L / 2
// rounded up to whole waves).
template <int kRows>
__global__ __launch_bounds__(kJT) void jacobi_svd_kernel(const double* R, int l, double tol, double* d, double* W) {
  constexpr int kLd = kLdJ;
  __shared__ double M[kMaxL * kLd];
  __shared__ double nrm2[kMaxL];
  const int nt = blockDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = nt / 64;
  const int L = l + (l & 1);   // even player count (a dummy column when l is odd)
  const int npairs = L / 2;
  const int rows = kRows * kJSub;
  for (int idx = tid; idx < L * rows; idx += nt) {
    const int j = idx / rows, i = idx - j * rows;
    M[j * kLd + i] = (j < l && i < l) ? R[(size_t)j * l + i] : 0.0;  // column j of R^T = row j of R
  }
  const int pi = tid / kJSub, sub = tid % kJSub;
  __syncthreads();
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    int rotated = 0;
    for (int r = 0; r < L - 1; ++r) {
      if (pi < npairs) {  // the same for the eight lanes of a group
        int p = r, q = L - 1;
        if (pi > 0) {
          p = r + pi;
          if (p >= L - 1) p -= L - 1;
          q = r - pi;
          if (q < 0) q += L - 1;
        }
        double x[kRows], y[kRows];
        double sa = 0.0, sb = 0.0, sg = 0.0;
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
          x[u] = M[p * kLd + sub + u * kJSub];
          y[u] = M[q * kLd + sub + u * kJSub];
        }
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
          sa = fma(x[u], x[u], sa);
          sb = fma(y[u], y[u], sb);
          sg = fma(x[u], y[u], sg);
        }
        sa = sum8(sa);
        sb = sum8(sb);
        sg = sum8(sg);
        // |g| > tol sqrt(a) sqrt(b), with the hardware estimates of 1 / sqrt (a threshold
        // needs no refinement; taken apart because a b underflows for columns near 1e-160).
        // Inner products below 1e-300 (subnormal 2 g) are left alone.
        if (fabs(sg) > 1e-300 && fabs(sg) * (__builtin_amdgcn_rsq(sa) * __builtin_amdgcn_rsq(sb)) > tol) {
          rotated = 1;
          // the smaller root t of t^2 + 2 zeta t - 1 = 0 (zeta is a ratio: no under- or
          // overflow from the scale of the columns); sqrt(1 + zeta^2) rounds to |zeta| beyond 1e8
          const double zeta = (sb - sa) * rcp_nr(2.0 * sg);
          const double az = fabs(zeta);
          const double zc = fmin(az, 1e8);
          const double w = fma(zc, zc, 1.0);
          const double root = az >= 1e8 ? az : w * rsq_nr(w);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(az + root);
          const double c = rsq_nr(fma(t, t, 1.0));
          const double sn = c * t;
#pragma unroll
          for (int u = 0; u < kRows; ++u) {
            M[p * kLd + sub + u * kJSub] = c * x[u] - sn * y[u];
            M[q * kLd + sub + u * kJSub] = sn * x[u] + c * y[u];
          }
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
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
  if (l > 0) small_matmul_kernel<<<l, kMaxL, 0, st>>>(A, B, l, C);
}

void launch_jacobi_svd(const double* R, int l, double tol, double* d, double* W, hipStream_t st) {
  if (l <= 0 || l > kMaxL) return;
  const int L = l + (l & 1);
  const int threads = (L / 2 * kJSub + 63) / 64 * 64;
  if (l <= 16) jacobi_svd_kernel<2><<<1, threads, 0, st>>>(R, l, tol, d, W);
  else if (l <= 32) jacobi_svd_kernel<4><<<1, threads, 0, st>>>(R, l, tol, d, W);
  else if (l <= 64) jacobi_svd_kernel<8><<<1, threads, 0, st>>>(R, l, tol, d, W);
  else jacobi_svd_kernel<16><<<1, threads, 0, st>>>(R, l, tol, d, W);
}

}  // namespace frpca
