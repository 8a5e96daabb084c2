// Symmetric eigendecomposition of the l x l Gram matrix (Alg. 2 step 2) and the small
// epilogues of eigSVD (steps 3-5) and of the final steps of Alg. 5/6.
//
// Eigensolver: cyclic two-sided Jacobi with the parallel round-robin ordering (each round
// pairs every index once; N-1 rounds make a sweep), in FP64, one workgroup of 16 waves. The
// upper triangle of G lives in LDS. A round first computes the N/2 rotations (Golub & Van
// Loan, sym.schur2: tau = (a_qq - a_pp)/(2 a_pq), t = sign(tau)/(|tau| + sqrt(1+tau^2))),
// then every 2x2 block between two pairs is rotated from both sides by one thread, while the
// eigenvector matrix V (V <- V J) is updated in registers: wave w holds rows 8w..8w+7, lane
// i holds the two columns of pair slot i. From one round to the next every index of slot
// i >= 1 advances by one (mod N-1) and slot 0 keeps N-1, so the columns move between
// neighbouring lanes (DPP wave shifts): a-columns shift down one lane (the last slot takes its
// own b-column), b-columns shift up one lane (slot 1 takes slot 0's b, slot 0 takes slot 1's
// a). A rotation is skipped when |a_pq| <= 1e-14 sqrt(a_pp a_qq) (relative test, so small
// eigenvalues keep full relative accuracy); sweeps stop when a whole sweep skips everything.
// Eigenvalues come out ascending (the order Alg. 2 and ind = k+s:-1:s+1 rely on), ties in
// index order.
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kEigThreads = 1024;
constexpr int kVRows = 8;  // rows of V per wave (16 waves x 8 = 128)
constexpr int kMaxSweeps = 40;
constexpr double kJacobiTol = 1e-14;
constexpr int kMaxN = kMaxL;  // even-padded size

__device__ __forceinline__ int packed(int i, int j, int n) {
  // upper-triangular row-major packing, i <= j
  return i * n - (i * (i - 1)) / 2 + (j - i);
}
__device__ __forceinline__ int pidx(int a, int b, int n) { return a <= b ? packed(a, b, n) : packed(b, a, n); }

// lane i <- lane i+1 (0x130) and lane i <- lane i-1 (0x138), per 32-bit half
__device__ __forceinline__ double from_next_lane(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_prev_lane(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Indices of round-robin slot x at round 0; each round every index of a slot x >= 1 and the
// second index of slot 0 advance by one modulo N-1.
__device__ __forceinline__ void slot_start(int x, int N, int& a, int& b) {
  if (x == 0) {
    a = N - 1;
    b = 0;
  } else {
    a = x;
    b = N - 1 - x;
  }
}
__device__ __forceinline__ int adv(int v, int N) { return (v + 1 == N - 1) ? 0 : v + 1; }
__device__ __forceinline__ void slot_advance(int x, int N, int& a, int& b) {
  if (x != 0) a = adv(a, N);
  b = adv(b, N);
}

__global__ __launch_bounds__(kEigThreads) void jacobi_kernel(const double* G, int ldg, int l, double* d_out,
                                                             double* W, int* nsweeps) {
  __shared__ double A[kMaxN * (kMaxN + 1) / 2];
  __shared__ double2 rot[kMaxN / 2];
  __shared__ double diag[kMaxN];
  __shared__ int rank_s[kMaxN];
  __shared__ int any_rot;
  const int N = l + (l & 1);  // an odd size gets a zero dummy index that never rotates
  const int half = N / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = 0; i < N; ++i)
    for (int j = i + tid; j < N; j += kEigThreads)
      A[packed(i, j, N)] = (i < l && j < l) ? G[(size_t)i * ldg + j] : 0.0;
  // my (at most two) off-diagonal blocks (i < j) of pair slots and their current indices
  const int nblk = half * (half - 1) / 2;
  int bi[2], bj[2], ai[2], bbi[2], aj[2], bbj[2];
  bool has[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int b = tid + u * kEigThreads;
    has[u] = b < nblk;
    int i = 0, r = has[u] ? b : 0;
    while (r >= half - 1 - i) {
      r -= half - 1 - i;
      ++i;
    }
    bi[u] = i;
    bj[u] = i + 1 + r;
    slot_start(bi[u], N, ai[u], bbi[u]);
    slot_start(bj[u], N, aj[u], bbj[u]);
  }
  // my pair slot (= lane) for the rotation (wave 0) and for V (all waves)
  int sa, sb;
  slot_start(lane, N, sa, sb);
  const bool live = lane < half;
  double va[kVRows], vb[kVRows];
#pragma unroll
  for (int k = 0; k < kVRows; ++k) {
    const int r = kVRows * wave + k;
    va[k] = (live && sa == r && r < l) ? 1.0 : 0.0;
    vb[k] = (live && sb == r && r < l) ? 1.0 : 0.0;
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int s = 0; s < N - 1; ++s) {
      if (tid < half) {
        const int p = min(sa, sb), q = max(sa, sb);
        const int ipp = packed(p, p, N), iqq = packed(q, q, N), ipq = packed(p, q, N);
        const double app = A[ipp], aqq = A[iqq], apq = A[ipq];
        double c = 1.0, sn = 0.0;
        if (apq != 0.0 && fabs(apq) > kJacobiTol * sqrt(fabs(app * aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
          A[ipp] = app - t * apq;
          A[iqq] = aqq + t * apq;
          A[ipq] = 0.0;
          any_rot = 1;
        }
        rot[tid] = make_double2(c, sn);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (has[u]) {
          const double2 ri = rot[bi[u]], rj = rot[bj[u]];
          if (ri.y != 0.0 || rj.y != 0.0) {
            const int p = min(ai[u], bbi[u]), q = max(ai[u], bbi[u]);
            const int r = min(aj[u], bbj[u]), t = max(aj[u], bbj[u]);
            const int ipr = pidx(p, r, N), ipt = pidx(p, t, N), iqr = pidx(q, r, N), iqt = pidx(q, t, N);
            const double gpr = A[ipr], gpt = A[ipt], gqr = A[iqr], gqt = A[iqt];
            // rows: (J_i^T G)
            const double xr = ri.x * gpr - ri.y * gqr, yr = ri.y * gpr + ri.x * gqr;
            const double xt = ri.x * gpt - ri.y * gqt, yt = ri.y * gpt + ri.x * gqt;
            // columns: (. J_j)
            A[ipr] = rj.x * xr - rj.y * xt;
            A[ipt] = rj.y * xr + rj.x * xt;
            A[iqr] = rj.x * yr - rj.y * yt;
            A[iqt] = rj.y * yr + rj.x * yt;
          }
        }
      }
      // V <- V J on this wave's rows, then move the columns to next round's slots
      {
        const double2 rr = live ? rot[lane] : make_double2(1.0, 0.0);
        const bool aq = sa < sb;
#pragma unroll
        for (int k = 0; k < kVRows; ++k) {
          if (rr.y != 0.0) {
            const double vp = aq ? va[k] : vb[k], vq = aq ? vb[k] : va[k];
            const double np = rr.x * vp - rr.y * vq, nq = rr.y * vp + rr.x * vq;
            va[k] = aq ? np : nq;
            vb[k] = aq ? nq : np;
          }
          if (half > 1) {
            const double t1 = from_next_lane(va[k]);
            const double t2 = from_prev_lane(vb[k]);
            const double na = (lane == 0) ? va[k] : (lane == half - 1 ? vb[k] : t1);
            const double nb = (lane == 0) ? t1 : t2;
            va[k] = na;
            vb[k] = nb;
          }
        }
      }
      slot_advance(lane, N, sa, sb);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        slot_advance(bi[u], N, ai[u], bbi[u]);
        slot_advance(bj[u], N, aj[u], bbj[u]);
      }
      __syncthreads();
    }
    if (!any_rot) break;
    __syncthreads();
  }
  if (tid == 0) *nsweeps = sweep + 1;
  // eigenvalues in ascending order, ties by index
  if (tid < l) diag[tid] = A[packed(tid, tid, N)];
  __syncthreads();
  if (tid < l) {
    const double v = diag[tid];
    int r = 0;
    for (int j = 0; j < l; ++j) {
      const double u = diag[j];
      r += (u < v) || (u == v && j < tid);
    }
    rank_s[tid] = r;
    d_out[r] = v;
  }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int k = 0; k < kVRows; ++k) {
      const int r = kVRows * wave + k;
      if (r < l) {
        if (sa < l) W[(size_t)r * l + rank_s[sa]] = va[k];
        if (sb < l) W[(size_t)r * l + rank_s[sb]] = vb[k];
      }
    }
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

// One block per column i: reduce the per-block candidates (|v|, row) in block order (ties:
// lowest row), then fold the sign into column i of Blong.
__global__ __launch_bounds__(256) void sign_final_kernel(const float* V, int k, int nblk, const float* pv,
                                                         const int* pr, float* sgn, double* Blong, int ldb, int l) {
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
    for (int a = t; a < l; a += 256) Blong[(size_t)a * ldb + i] = -Blong[(size_t)a * ldb + i];
}

__global__ __launch_bounds__(256) void sign_apply_kernel(float* V, int64_t rows, int k, const float* sgn) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * k) return;
  const int i = (int)(idx % k);
  if (sgn[i] < 0.0f) V[idx] = -V[idx];
}

}  // namespace

void launch_eig(const double* G, int ldg, int l, double* d, double* W, int* nsweeps, hipStream_t st) {
  jacobi_kernel<<<1, kEigThreads, 0, st>>>(G, ldg, l, d, W, nsweeps);
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
  sign_final_kernel<<<k, 256, 0, st>>>(V, k, (int)nblk, pv, pr, sgn, Blong, ldb, brows);
  sign_apply_kernel<<<(unsigned)((rows * k + 255) / 256), 256, 0, st>>>(V, rows, k, sgn);
}

}  // namespace frpca
