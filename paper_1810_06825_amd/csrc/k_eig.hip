// Symmetric eigendecomposition of the l x l Gram matrix (Alg. 2 step 2) and the small
// epilogues of eigSVD (steps 3-5) and of the final steps of Alg. 5/6.
//
// Eigensolver: cyclic two-sided Jacobi with the parallel round-robin ordering (each round
// pairs every index once; l-1 rounds make a sweep), in FP64, one workgroup. The upper
// triangle of G lives in LDS; a round first computes the l/2 rotations (Golub & Van Loan,
// sym.schur2: tau = (a_qq - a_pp)/(2 a_pq), t = sign(tau)/(|tau| + sqrt(1+tau^2))), then
// every 2x2 block between two pairs is rotated from both sides by one thread. A rotation is
// skipped when |a_pq| <= 1e-14 sqrt(a_pp a_qq) (relative test, so small eigenvalues keep
// full relative accuracy); sweeps stop when a whole sweep skips everything. Rotations are
// logged, and a second kernel rebuilds each row of the eigenvector matrix by replaying the
// log, so G and W never need to share the LDS. Eigenvalues come out ascending (the order
// Alg. 2 and ind = k+s:-1:s+1 rely on), ties in index order.
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kEigThreads = 1024;
constexpr int kMaxSweeps = 40;
constexpr double kJacobiTol = 1e-14;
constexpr int kMaxN = kMaxL;  // even-padded size

__device__ __forceinline__ int packed(int i, int j, int n) {
  // upper-triangular row-major packing, i <= j
  return i * n - (i * (i - 1)) / 2 + (j - i);
}
__device__ __forceinline__ int pidx(int a, int b, int n) { return a <= b ? packed(a, b, n) : packed(b, a, n); }

// Round-robin pair `slot` of round s for N (even) indices.
__device__ __forceinline__ void rr_pair(int s, int slot, int N, int& p, int& q) {
  int a, b;
  if (slot == 0) {
    a = N - 1;
    b = s;
  } else {
    a = (s + slot) % (N - 1);
    b = (s - slot + (N - 1)) % (N - 1);
  }
  p = min(a, b);
  q = max(a, b);
}

__global__ __launch_bounds__(kEigThreads) void jacobi_kernel(const double* G, int ldg, int l, double* rotlog,
                                                             int* nsteps, double* diag_out) {
  __shared__ double A[kMaxN * (kMaxN + 1) / 2];
  __shared__ double rc[kMaxN / 2], rs[kMaxN / 2];
  __shared__ int rflag[kMaxN / 2];
  __shared__ unsigned short pairs[(kMaxN - 1) * (kMaxN / 2)];  // p | q << 8 for (round, slot)
  __shared__ int rowbase[kMaxN];                               // packed(a, b) = rowbase[a] + b, a <= b
  __shared__ unsigned char blk_i[kMaxN / 2 * (kMaxN / 2 - 1) / 2], blk_j[kMaxN / 2 * (kMaxN / 2 - 1) / 2];
  __shared__ int any_rot;
  const int N = l + (l & 1);  // an odd size gets a zero dummy index that never rotates
  const int half = N / 2;
  const int tid = threadIdx.x;
  for (int a = tid; a < N; a += kEigThreads) rowbase[a] = a * N - (a * (a - 1)) / 2 - a;
  for (int i = 0; i < N; ++i)
    for (int j = i + tid; j < N; j += kEigThreads)
      A[packed(i, j, N)] = (i < l && j < l) ? G[(size_t)i * ldg + j] : 0.0;
  for (int e = tid; e < (N - 1) * half; e += kEigThreads) {
    int p, q;
    rr_pair(e / half, e % half, N, p, q);
    pairs[e] = (unsigned short)(p | (q << 8));
  }
  const int nblk = half * (half - 1) / 2;
  for (int b = tid; b < nblk; b += kEigThreads) {
    int i = 0, r = b;
    while (r >= half - 1 - i) {
      r -= half - 1 - i;
      ++i;
    }
    blk_i[b] = (unsigned char)i;
    blk_j[b] = (unsigned char)(i + 1 + r);
  }
  __syncthreads();
  auto pk = [&](int a, int b) { return a <= b ? rowbase[a] + b : rowbase[b] + a; };
  int step = 0;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int s = 0; s < N - 1; ++s, ++step) {
      const unsigned short* pr = pairs + s * half;
      if (tid < half) {
        const int p = pr[tid] & 255, q = pr[tid] >> 8;
        const int ipp = rowbase[p] + p, iqq = rowbase[q] + q, ipq = rowbase[p] + q;
        const double app = A[ipp], aqq = A[iqq], apq = A[ipq];
        double c = 1.0, sn = 0.0;
        int f = 0;
        if (apq != 0.0 && fabs(apq) > kJacobiTol * sqrt(fabs(app * aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
          A[ipp] = app - t * apq;
          A[iqq] = aqq + t * apq;
          A[ipq] = 0.0;
          f = 1;
          any_rot = 1;
        }
        rc[tid] = c;
        rs[tid] = sn;
        rflag[tid] = f;
        rotlog[((size_t)step * (kMaxN / 2) + tid) * 2 + 0] = c;
        rotlog[((size_t)step * (kMaxN / 2) + tid) * 2 + 1] = sn;
      }
      __syncthreads();
      for (int b = tid; b < nblk; b += kEigThreads) {
        const int i = blk_i[b], j = blk_j[b];
        if (!(rflag[i] | rflag[j])) continue;
        const int p = pr[i] & 255, q = pr[i] >> 8, r = pr[j] & 255, t = pr[j] >> 8;
        const double ci = rc[i], si = rs[i], cj = rc[j], sj = rs[j];
        const int ipr = pk(p, r), ipt = pk(p, t), iqr = pk(q, r), iqt = pk(q, t);
        const double gpr = A[ipr], gpt = A[ipt], gqr = A[iqr], gqt = A[iqt];
        // rows: (J_i^T G)
        const double xr = ci * gpr - si * gqr, yr = si * gpr + ci * gqr;
        const double xt = ci * gpt - si * gqt, yt = si * gpt + ci * gqt;
        // columns: (. J_j)
        A[ipr] = cj * xr - sj * xt;
        A[ipt] = sj * xr + cj * xt;
        A[iqr] = cj * yr - sj * yt;
        A[iqt] = sj * yr + cj * yt;
      }
      __syncthreads();
    }
    if (!any_rot) break;
    __syncthreads();
  }
  if (tid == 0) *nsteps = step;
  for (int i = tid; i < l; i += kEigThreads) diag_out[i] = A[rowbase[i] + i];
}

// Eigenvalues in ascending order (ties by index) and the rank of each original index.
__global__ __launch_bounds__(128) void eig_sort_kernel(const double* diag, int l, double* d, int* rank) {
  const int i = threadIdx.x;
  if (i >= l) return;
  const double v = diag[i];
  int r = 0;
  for (int j = 0; j < l; ++j) {
    const double u = diag[j];
    r += (u < v) || (u == v && j < i);
  }
  rank[i] = r;
  d[r] = v;
}

// Row `blockIdx.x` of the eigenvector matrix: e_r^T J_1 J_2 ... J_T, replayed from the log
// by one wave with the row in registers. Lane i holds the two entries of round-robin slot i
// (indices ia, ib). From one round to the next every index of slot i >= 1 advances by one
// (mod N-1) and slot 0 keeps N-1, which moves the values between neighbouring lanes:
// a-values shift down one lane (the last slot takes its own b-value), b-values shift up one
// lane (slot 1 takes slot 0's b, slot 0 takes slot 1's a).
__global__ __launch_bounds__(64) void eigvec_kernel(const double* rotlog, const int* nsteps, int l, const int* rank,
                                                    double* W) {
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  const int N = l + (l & 1), half = N / 2;
  const bool live = lane < half;
  int ia, ib;
  if (lane == 0) {
    ia = N - 1;
    ib = 0;
  } else {
    ia = lane;
    ib = N - 1 - lane;
  }
  double va = (ia == r) ? 1.0 : 0.0, vb = (ib == r) ? 1.0 : 0.0;
  const int T = *nsteps;
  constexpr int kPre = 8;
  double cb[kPre], sb[kPre], cn[kPre], sn[kPre];
  auto fetch = [&](int st0, double* c, double* s) {
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      c[u] = 1.0;
      s[u] = 0.0;
      if (live && st0 + u < T) {
        c[u] = rotlog[((size_t)(st0 + u) * (kMaxN / 2) + lane) * 2 + 0];
        s[u] = rotlog[((size_t)(st0 + u) * (kMaxN / 2) + lane) * 2 + 1];
      }
    }
  };
  fetch(0, cb, sb);
  const int up = min(lane + 1, 63), dn = max(lane - 1, 0);
  for (int st0 = 0; st0 < T; st0 += kPre) {
    fetch(st0 + kPre, cn, sn);  // next batch in flight while this one is applied
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      if (st0 + u < T) {
        if (sb[u] != 0.0) {
          // the logged rotation is for (p, q) = (min, max) of the slot's indices
          const bool aq = ia < ib;
          const double vp = aq ? va : vb, vq = aq ? vb : va;
          const double np = cb[u] * vp - sb[u] * vq, nq = sb[u] * vp + cb[u] * vq;
          va = aq ? np : nq;
          vb = aq ? nq : np;
        }
        if (half > 1) {  // with a single pair nothing moves
          const double t1 = __shfl(va, up);
          const double t2 = __shfl(vb, dn);
          const double na = (lane == 0) ? va : (lane == half - 1 ? vb : t1);
          const double nb = (lane == 0) ? t1 : t2;
          va = na;
          vb = nb;
        }
        if (lane != 0) ia = (ia + 1 == N - 1) ? 0 : ia + 1;
        ib = (ib + 1 == N - 1) ? 0 : ib + 1;
      }
    }
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      cb[u] = cn[u];
      sb[u] = sn[u];
    }
  }
  if (live) {
    if (ia < l) W[(size_t)r * l + rank[ia]] = va;
    if (ib < l) W[(size_t)r * l + rank[ib]] = vb;
  }
}

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
                                                           float* S, int* ndropped) {
  const double smax = sqrt(fmax(d[l - 1], 0.0));
  for (int idx = threadIdx.x; idx < l * ldb; idx += blockDim.x) {
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
  if (threadIdx.x == 0) {
    int nd = 0;
    for (int i = 0; i < k; ++i) {
      const double s = sqrt(fmax(d[l - 1 - i], 0.0));
      const bool keep = s > rank_tol * smax && s > 0.0;
      S[i] = keep ? (float)s : 0.0f;
      nd += !keep;
    }
    *ndropped = nd;
  }
}

// Sign convention: per column i of V (rows x k, ld k), the largest |entry| (ties: lowest
// row). Pass 1: one partial (|v|, row) per block and column; pass 2 reduces in block order.
constexpr int kSignRows = 256;

__global__ __launch_bounds__(256) void sign_partial_kernel(const float* V, int64_t rows, int k, float* pv, int* pr) {
  const int64_t r0 = (int64_t)blockIdx.x * kSignRows;
  const int64_t r1 = min(rows, r0 + kSignRows);
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    float best = -1.0f;
    int brow = 0;
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

__global__ __launch_bounds__(128) void sign_final_kernel(const float* V, int k, int nblk, const float* pv,
                                                         const int* pr, float* sgn, double* Blong, int ldb, int l) {
  const int i = threadIdx.x;
  if (i >= k) return;
  float best = -1.0f;
  int brow = 0;
  for (int b = 0; b < nblk; ++b) {
    const float a = pv[(size_t)b * k + i];
    if (a > best) {
      best = a;
      brow = pr[(size_t)b * k + i];
    }
  }
  const float s = (V[(size_t)brow * k + i] < 0.0f) ? -1.0f : 1.0f;
  sgn[i] = s;
  if (s < 0.0f)
    for (int a = 0; a < l; ++a) Blong[(size_t)a * ldb + i] = -Blong[(size_t)a * ldb + i];
}

__global__ __launch_bounds__(256) void sign_apply_kernel(float* V, int64_t rows, int k, const float* sgn) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * k) return;
  const int i = (int)(idx % k);
  if (sgn[i] < 0.0f) V[idx] = -V[idx];
}

}  // namespace

size_t eig_log_bytes(int /*l*/) { return (size_t)kMaxSweeps * (kMaxN - 1) * (kMaxN / 2) * 2 * sizeof(double); }

void launch_eig(const double* G, int ldg, int l, double* d, double* W, double* rotlog, int* nsteps, int* order,
                double* diag_tmp, hipStream_t st) {
  jacobi_kernel<<<1, kEigThreads, 0, st>>>(G, ldg, l, rotlog, nsteps, diag_tmp);
  eig_sort_kernel<<<1, 128, 0, st>>>(diag_tmp, l, d, order);
  eigvec_kernel<<<l, 64, 0, st>>>(rotlog, nsteps, l, order, W);
}

void launch_eigsvd_coeffs(const double* d, const double* W, int l, int ldb, double tol, double* B, double* sigma,
                          hipStream_t st) {
  const int total = l * ldb;
  eigsvd_coeffs_kernel<<<(total + 255) / 256, 256, 0, st>>>(d, W, l, ldb, tol, B, sigma);
}

void launch_final_coeffs(const double* d, const double* W, int l, int k, int ldb, double rank_tol, double* Blong,
                         double* Bshort, float* S, int* ndropped, hipStream_t st) {
  final_coeffs_kernel<<<1, 256, 0, st>>>(d, W, l, k, ldb, rank_tol, Blong, Bshort, S, ndropped);
}

size_t sign_partial_bytes(int64_t rows, int k) {
  const int64_t nblk = (rows + kSignRows - 1) / kSignRows;
  return (size_t)nblk * k * (sizeof(float) + sizeof(int)) + (size_t)k * sizeof(float) + 256;
}

void launch_sign_fix(float* V, int64_t rows, int k, double* Blong, int ldb, int brows, void* partial,
                     hipStream_t st) {
  const int64_t nblk = (rows + kSignRows - 1) / kSignRows;
  float* pv = static_cast<float*>(partial);
  int* pr = reinterpret_cast<int*>(pv + nblk * k);
  float* sgn = reinterpret_cast<float*>(pr + nblk * k);
  sign_partial_kernel<<<(unsigned)nblk, 256, 0, st>>>(V, rows, k, pv, pr);
  sign_final_kernel<<<1, 128, 0, st>>>(V, k, (int)nblk, pv, pr, sgn, Blong, ldb, brows);
  sign_apply_kernel<<<(unsigned)((rows * k + 255) / 256), 256, 0, st>>>(V, rows, k, sgn);
}

}  // namespace frpca
