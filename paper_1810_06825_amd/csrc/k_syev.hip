// Symmetric eigendecomposition of the l x l Gram matrix (Alg. 2 step 2), FP64, in three
// kernels: phases 1-2 and phases 4-5 each on one workgroup of 16 waves, phase 3 on one wave per
// eigenvalue across the chip. Householder tridiagonalization, then eigenpairs of the
// tridiagonal T by the multiple relatively robust representations idea (Dhillon & Parlett,
// 2004), then the back-transformation:
//
//  1. Q^T G Q = T by Householder reflectors H_k = I - tau_k v_k v_k^T, v_k(0) = 1 (Golub &
//     Van Loan, Alg. 8.3.1). G lives in registers as 4 x 4 tiles (thread t holds rows
//     4 (t / 32).., columns 4 (t % 32)..), so sums over a row are half-wave DPP reductions.
//     Step k takes two barriers: one after v_k and the partial products p = tau A22 v, one
//     after the rank-2 update A22 -= v w^T + w v^T, w = p - (tau p.v / 2) v, during which the
//     owners of column k + 1 also reduce its norm for the next step. Waves whose tiles lie
//     wholly in the finished part skip the work. The v_k stay in LDS during the phase and
//     then go to a global scratch buffer for step 5.
//  2. T splits where |e_j| <= eps ||T||. Each unreduced block gets a root representation
//     L D L^T = T - sigma I with every D_i > 0. For a Gram matrix sigma = -nb eps ||T_b||
//     works; otherwise sigma is the smallest eigenvalue (multisection on Sturm counts of T)
//     minus a margin that grows until D > 0. A positive definite L D L^T determines its
//     eigenvalues to high relative accuracy, so eigenvectors of eigenvalues with a relative
//     gap of 1e-3 or more come out numerically orthogonal without any reorthogonalization.
//  3. Eigenvalues mu of L D L^T by multisection on negative-pivot counts of the stationary
//     qd transform L D L^T - x I = L+ D+ L+^T (a wave per eigenvalue, 65 subintervals per
//     step, geometric points while the bracket spans a wide ratio, reciprocals by the
//     hardware estimate and two Newton steps), to a relative width of 4 eps.
//  4. Each isolated eigenvector from the twisted factorization of L D L^T - mu I at the index
//     r where |gamma_r| = |s_r + p_r + mu| is smallest (stationary and progressive qd
//     transforms): z_r = 1, z_i = -L+_i z_i+1 above r, z_i+1 = -U-_i z_i below r. Eigenvalues
//     with a relative gap under 1e-3 form clusters; their vectors start from the twisted
//     ones (slightly perturbed) and take three steps of inverse iteration with shifts kept
//     10 eps apart, each followed by Gram-Schmidt (twice) against the earlier members.
//  5. W = H_0 H_1 ... H_{n-3} Z with Z in registers (each wave owns eight columns) and the
//     reflectors staged in LDS, so every wave applies all of them to its own columns with no
//     barrier; eigenvalues sorted ascending (the order Alg. 2 and the final selection
//     ind = k+s:-1:s+1 rely on; ties in index order).
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kT = 1024;             // threads
constexpr int kS = kMaxL + 1;        // odd LDS row stride (doubles)
constexpr double kEps = 2.220446049250313e-16;
constexpr double kMinRelGap = 1e-3;  // relative gap below which eigenvalues form a cluster
constexpr int kClusterIters = 3;
constexpr int kLdsSlots = 10;        // clustered columns whose L+ factors stay in LDS

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum over all threads of the workgroup, every thread gets it (two barriers).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kT / 64; ++w) s += red[w];
  return s;
}

// Lane l's value, broadcast to the wave (l uniform).
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// DPP move of a double (both halves through the same control); lanes whose source is invalid
// or whose row is masked off read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over each half-wave (lanes 0-31, 32-63), valid in lanes 31 and 63: row shifts 1, 2, 4, 8
// put each row's sum in its lane 15, then row 0's (row 2's) total is broadcast into row 1 (3).
__device__ __forceinline__ double half_sum_to_last(double v) {
  v += dpp64<0x111, 0xF>(v);
  v += dpp64<0x112, 0xF>(v);
  v += dpp64<0x114, 0xF>(v);
  v += dpp64<0x118, 0xF>(v);
  v += dpp64<0x142, 0xA>(v);
  return v;
}

// Sum over each group of 8 lanes, in all 8: quad xor 1, quad xor 2, then lane i + lane 7 - i.
__device__ __forceinline__ double oct_allsum(double v) {
  v += dpp64<0xB1, 0xF>(v);
  v += dpp64<0x4E, 0xF>(v);
  v += dpp64<0x141, 0xF>(v);
  return v;
}

// 1/v to within a few ulps: hardware reciprocal refined by two Newton steps (cheaper than the
// IEEE division sequence on the serial chains below).
__device__ __forceinline__ double rcp2(double v) {
  double r = __builtin_amdgcn_rcp(v);
  r = fma(fma(-v, r, 1.0), r, r);
  return fma(fma(-v, r, 1.0), r, r);
}

__device__ __forceinline__ double guard(double v, double pivmin) {
  return fabs(v) < pivmin ? -pivmin : v;
}

// Number of eigenvalues of T[o, o+nb) below x (LDL^T recurrence of T - x I).
__device__ int sturm_T(const double* d, const double* e2, int o, int nb, double x, double pivmin) {
  double q = guard(d[o] - x, pivmin);
  int c = q < 0.0;
  for (int j = 1; j < nb; ++j) {
    q = guard((d[o + j] - x) - e2[o + j - 1] / q, pivmin);
    c += q < 0.0;
  }
  return c;
}

// Number of eigenvalues of L D L^T (block [o, o+nb)) below x: negative pivots of the
// stationary qd transform. Four steps at a time with their LDS operands fetched first, so the
// dependent chain does not wait on loads.
__device__ __forceinline__ void negstep(double& s, int& c, double Di, double LLDi, double x, double pivmin) {
  const double dp = guard(Di + s, pivmin);
  c += dp < 0.0;
  // 1/dp by the hardware reciprocal and two Newton steps (a few ulps at most: the count is
  // backward stable under such relative perturbations of the representation)
  s = (s * rcp2(dp)) * LLDi - x;
}

__device__ int negcount(const double* D, const double* LLD, int o, int nb, double x, double pivmin) {
  double s = -x;
  int c = 0;
  const int end = o + nb - 1;
  int i = o;
  for (; i + 4 <= end; i += 4) {
    double d4[4], l4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      d4[u] = D[i + u];
      l4[u] = LLD[i + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) negstep(s, c, d4[u], l4[u], x, pivmin);
  }
  for (; i < end; ++i) negstep(s, c, D[i], LLD[i], x, pivmin);
  c += guard(D[end] + s, pivmin) < 0.0;
  return c;
}

// Deterministic perturbation in [-1, 1) for the start vectors of clustered eigenvalues.
__device__ __forceinline__ double jitter(int g, int i) {
  uint32_t h = (uint32_t)g * 0x9E3779B1u ^ ((uint32_t)i * 0x85EBCA77u + 0x165667B1u);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)h * (2.0 / 4294967296.0) - 1.0;
}

// The three kernels of one decomposition hand over through global scratch: the reflectors,
// the cluster solves' L+ columns, then these arrays (written by the first kernel, mu by the
// second).
struct EigState {
  double *d, *tau, *Dr, *Lr, *LLD, *bsig, *bgu, *btn, *mu, *misc;
  int *bstart, *bsize;
};
constexpr size_t kStateDoubles = 9 * kMaxL + 8;
__device__ __forceinline__ EigState eig_state(double* scratch) {
  double* b = scratch + 2 * kMaxL * kMaxL;
  EigState st;
  st.d = b;
  st.tau = b + kMaxL;
  st.Dr = b + 2 * kMaxL;
  st.Lr = b + 3 * kMaxL;
  st.LLD = b + 4 * kMaxL;
  st.bsig = b + 5 * kMaxL;
  st.bgu = b + 6 * kMaxL;
  st.btn = b + 7 * kMaxL;
  st.mu = b + 8 * kMaxL;
  st.misc = b + 9 * kMaxL;  // [0]: pivmin
  st.bstart = reinterpret_cast<int*>(b + kStateDoubles);
  st.bsize = st.bstart + kMaxL;
  return st;
}

// Phases 1 and 2.
__global__ __launch_bounds__(kT) void syev_tridiag_kernel(const double* G, int ldg, int n, double* scratch) {
  __shared__ double A[kMaxL * kS];  // rows hold the reflectors v_k during the phase
  __shared__ double d[kMaxL], e[kMaxL], e2[kMaxL], tau[kMaxL];
  __shared__ __align__(16) double pw[kMaxL];
  __shared__ double Dr[kMaxL], Lr[kMaxL], LLD[kMaxL];
  __shared__ double bsig[kMaxL], bgl[kMaxL], bgu[kMaxL], btn[kMaxL];
  __shared__ double red[kT / 64], red2[kT / 64];
  __shared__ __align__(16) double colbuf[kMaxL];
  __shared__ int bstart[kMaxL], bsize[kMaxL], bbad[kMaxL];
  __shared__ int sh_int[4];
  __shared__ double sh_dbl[4];
  double* house = scratch;                   // kMaxL x kMaxL reflectors
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // ---------------------------------------------------------------- 1. tridiagonalization
  // G in registers: thread t holds the 4 x 4 tile of rows 4 rb.., columns 4 cb.. (rb = t / 32,
  // cb = t % 32), so a wave holds two tile rows and a half-wave reduction sums over a row.
  const int rb = tid >> 5, cb = tid & 31;
  double ta[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int R = 4 * rb + a, C = 4 * cb + b;
      ta[a][b] = (R < n && C < n) ? G[(size_t)R * ldg + C] : 0.0;
    }
  // column 0 into colbuf, with its sum of squares below the subdiagonal (owners: cb == 0)
  {
    double part = 0.0;
    if (cb == 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int R = 4 * rb + a;
        colbuf[R] = ta[a][0];
        if (R >= 2 && R < n) part += ta[a][0] * ta[a][0];
      }
    }
    const double wpart = readlane_d(part, 0) + readlane_d(part, 32);
    if (lane == 0) red[wave] = wpart;
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    // waves whose two tile rows lie above the trailing block have nothing to do this step
    // (they stay idle from here on and contribute zeros to the reductions)
    const bool wact = 8 * wave + 7 >= k + 1;
    if (rb == (k >> 2) && cb == (k >> 2)) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (a == (k & 3)) d[k] = ta[a][a];
    }
    double vr[4], vc[4], K = 0.0;
    if (wact) {
      double sigma = 0.0;
#pragma unroll
      for (int w = 0; w < kT / 64; ++w) sigma += red[w];
      const double x0 = colbuf[k + 1];
      double tk = 0.0, beta = x0, scal = 0.0;
      if (sigma != 0.0) {
        const double mu0 = sqrt(x0 * x0 + sigma);
        beta = (x0 <= 0.0) ? mu0 : -mu0;
        tk = (beta - x0) * rcp2(beta);
        scal = rcp2(x0 - beta);
      }
      if (tid == kT - 64) {  // the last wave is never idle
        tau[k] = tk;
        e[k] = beta;
      }
      // the own four rows and four columns of the column come as 16-byte LDS reads shared by
      // all four selects (a read per element sits in its own branch and waits alone)
      const double2 r01 = *reinterpret_cast<const double2*>(colbuf + 4 * rb);
      const double2 r23 = *reinterpret_cast<const double2*>(colbuf + 4 * rb + 2);
      const double2 c01 = *reinterpret_cast<const double2*>(colbuf + 4 * cb);
      const double2 c23 = *reinterpret_cast<const double2*>(colbuf + 4 * cb + 2);
      const double xr[4] = {r01.x, r01.y, r23.x, r23.y}, xc[4] = {c01.x, c01.y, c23.x, c23.y};
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int R = 4 * rb + a, C = 4 * cb + a;
        vr[a] = (R == k + 1) ? 1.0 : ((R > k + 1 && R < n) ? xr[a] * scal : 0.0);
        vc[a] = (C == k + 1) ? 1.0 : ((C > k + 1 && C < n) ? xc[a] * scal : 0.0);
      }
      // v_k is kept in row k of the LDS matrix, which is free during this phase (a global
      // store here would make every barrier wait for it)
      if (cb == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int R = 4 * rb + a;
          if (R >= k + 1 && R < n) A[k * kS + (R - k - 1)] = vr[a];
        }
      }
      // p = tau A22 v on the own rows: partial over the own columns, summed over the half-wave
      double pp[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) acc += ta[a][b] * vc[b];
        pp[a] = half_sum_to_last(acc);
      }
      double pvp = 0.0;
      if (cb == 31) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int R = 4 * rb + a;
          if (R >= k + 1 && R < n) {
            const double pr = tk * pp[a];
            pw[R] = pr;
            pvp += pr * vr[a];
          }
        }
      }
      const double wpv = readlane_d(pvp, 31) + readlane_d(pvp, 63);
      if (lane == 0) red2[wave] = wpv;
      K = tk;
    } else if (lane == 0) {
      red2[wave] = 0.0;
    }
    __syncthreads();  // (A)
    if (wact) {
      double pv = 0.0;
#pragma unroll
      for (int w = 0; w < kT / 64; ++w) pv += red2[w];
      K *= 0.5 * pv;
      double wr[4], wc[4];
      const double2 p01 = *reinterpret_cast<const double2*>(pw + 4 * rb);
      const double2 p23 = *reinterpret_cast<const double2*>(pw + 4 * rb + 2);
      const double2 q01 = *reinterpret_cast<const double2*>(pw + 4 * cb);
      const double2 q23 = *reinterpret_cast<const double2*>(pw + 4 * cb + 2);
      const double pr4[4] = {p01.x, p01.y, p23.x, p23.y}, pc4[4] = {q01.x, q01.y, q23.x, q23.y};
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int R = 4 * rb + a, C = 4 * cb + a;
        wr[a] = (R >= k + 1 && R < n) ? pr4[a] - K * vr[a] : 0.0;
        wc[a] = (C >= k + 1 && C < n) ? pc4[a] - K * vc[a] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) ta[a][b] -= vr[a] * wc[b] + wr[a] * vc[b];
      // column k+1 into colbuf and the next step's sum of squares (owners: cb == (k+1)/4)
      const int cbn = (k + 1) >> 2, bn = (k + 1) & 3;
      double part = 0.0;
      if (cb == cbn) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if (b == bn) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const int R = 4 * rb + a;
              colbuf[R] = ta[a][b];
              if (R >= k + 3 && R < n) part += ta[a][b] * ta[a][b];
            }
          }
        }
      }
      const double wpart = readlane_d(part, cbn) + readlane_d(part, 32 + cbn);
      if (lane == 0) red[wave] = wpart;
    } else if (lane == 0) {
      red[wave] = 0.0;
    }
    __syncthreads();  // (B)
  }
  // the last 2 x 2 block
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int R = 4 * rb + a, C = 4 * cb + b;
      if (R == C && R >= n - 2 && R >= 0 && R < n) d[R] = ta[a][b];
      if (n >= 2 && R == n - 1 && C == n - 2) e[n - 2] = ta[a][b];
    }
  if (tid == 0) e[n - 1] = 0.0;
  __syncthreads();
  // the reflectors move to global scratch until the back-transformation
  for (int idx = tid; idx < (n - 2) * kMaxL; idx += kT) {
    const int k = idx / kMaxL, i = idx - k * kMaxL;
    if (i < n - k - 1) house[idx] = A[k * kS + i];
  }

  // ---------------------------------------------------------------- 2. blocks and root representations
  if (tid == 0) {
    double tn = 0.0;
    for (int j = 0; j < n; ++j) tn = fmax(tn, fmax(fabs(d[j]), fabs(e[j])));
    sh_dbl[0] = tn;
    int o = 0;
    for (int j = 0; j < n; ++j) {
      if (j + 1 == n || fabs(e[j]) <= kEps * tn) {
        e[j] = 0.0;
        double gl = 1e300, gu = -1e300, tb = 0.0;
        for (int t = o; t <= j; ++t) {
          const double r = (t > o ? fabs(e[t - 1]) : 0.0) + fabs(e[t]);
          gl = fmin(gl, d[t] - r);
          gu = fmax(gu, d[t] + r);
          tb = fmax(tb, fmax(fabs(d[t]), fabs(e[t])));
          bstart[t] = o;
          bsize[t] = j - o + 1;
        }
        bgl[o] = gl;
        bgu[o] = gu;
        btn[o] = tb;
        o = j + 1;
      }
    }
  }
  __syncthreads();
  const double tnorm = sh_dbl[0];
  const double pivmin = fmax(tnorm * tnorm * 1e-300, 1e-300);
  for (int j = tid; j < n; j += kT) e2[j] = e[j] * e[j];
  // factor L D L^T = T_b - sigma I with sigma = -nb eps ||T_b||: one thread per block
  if (tid < n && bstart[tid] == tid) {
    const int o = tid, nb = bsize[tid];
    int bad = 0;
    if (nb > 1) {
      const double sg = -(double)nb * kEps * btn[o];
      double Dc = d[o] - sg;
      for (int i = o; i < o + nb - 1; ++i) {
        bad |= !(Dc > 0.0);
        const double L = e[i] / Dc;
        Dr[i] = Dc;
        Lr[i] = L;
        LLD[i] = L * L * Dc;
        Dc = d[i + 1] - sg - L * e[i];
      }
      bad |= !(Dc > 0.0);
      Dr[o + nb - 1] = Dc;
      bsig[o] = sg;
    }
    bbad[o] = bad;
  }
  __syncthreads();
  // blocks that are not (numerically) positive semidefinite: shift from below the spectrum
  for (int o = 0; o < n; o += bsize[o]) {
    if (!bbad[o]) continue;  // uniform: LDS value read by every thread
    const int nb = bsize[o];
    double lo = bgl[o], hi = bgu[o];
    const double pad = 2.0 * kEps * fmax(fabs(lo), fabs(hi)) + pivmin;
    lo -= pad;
    hi += pad;
    for (int it = 0; it < 16; ++it) {
      if (hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi)) + 2.0 * pivmin) break;  // uniform
      const double x = lo + (hi - lo) * (double)(tid + 1) / (double)(kT + 1);
      const int c = sturm_T(d, e2, o, nb, x, pivmin);
      if (tid == 0) sh_int[0] = kT;
      __syncthreads();
      if (c >= 1) atomicMin(&sh_int[0], tid);
      __syncthreads();
      const int b = sh_int[0];
      const double nlo = (b == 0) ? lo : lo + (hi - lo) * (double)b / (double)(kT + 1);
      const double nhi = (b == kT) ? hi : lo + (hi - lo) * (double)(b + 1) / (double)(kT + 1);
      lo = nlo;
      hi = nhi;
      __syncthreads();
    }
    if (tid == 0) {
      double delta = (double)nb * kEps * fmax(btn[o], (bgu[o] - bgl[o]));
      for (int attempt = 0; attempt < 200; ++attempt) {
        const double sg = lo - delta;
        double Dc = d[o] - sg;
        bool ok = Dc > 0.0;
        for (int i = o; i < o + nb - 1 && ok; ++i) {
          const double L = e[i] / Dc;
          Dr[i] = Dc;
          Lr[i] = L;
          LLD[i] = L * L * Dc;
          Dc = d[i + 1] - sg - L * e[i];
          ok = Dc > 0.0;
        }
        if (ok) {
          Dr[o + nb - 1] = Dc;
          bsig[o] = sg;
          break;
        }
        delta *= 4.0;
      }
    }
    __syncthreads();
  }

  // hand-over to the eigenvalue and eigenvector kernels
  const EigState st = eig_state(scratch);
  for (int j = tid; j < n; j += kT) {
    st.d[j] = d[j];
    st.tau[j] = tau[j];
    st.Dr[j] = Dr[j];
    st.Lr[j] = Lr[j];
    st.LLD[j] = LLD[j];
    st.bsig[j] = bsig[j];
    st.bgu[j] = bgu[j];
    st.btn[j] = btn[j];
    st.bstart[j] = bstart[j];
    st.bsize[j] = bsize[j];
  }
  if (tid == 0) st.misc[0] = pivmin;
}

// Phase 3: one wave per eigenvalue, multisection over 65 subintervals per step (lane i takes
// the (i+1)-th point; geometric points while the bracket spans a wide ratio, or powers of two
// below hi while its lower end is still 0), down to a relative width of 4 eps. Each lane runs
// one negative-pivot count, a serial chain of n steps, so a step of the search costs one
// chain; the waves of all eigenvalues run on separate SIMDs.
constexpr int kBisWaves = 4;
__global__ __launch_bounds__(64 * kBisWaves) void syev_bisect_kernel(int n, double* scratch) {
  __shared__ double Ds[kMaxL], Ls[kMaxL];
  const EigState st = eig_state(scratch);
  for (int j = threadIdx.x; j < n; j += 64 * kBisWaves) {
    Ds[j] = st.Dr[j];
    Ls[j] = st.LLD[j];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int g = blockIdx.x * kBisWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (g >= n) return;
  const int o = st.bstart[g], nb = st.bsize[g];
  if (nb <= 1) {
    if (lane == 0) st.mu[g] = 0.0;
    return;
  }
  const double pivmin = st.misc[0];
  const int want = g - o;
  double lo = 0.0;
  double hi = (st.bgu[o] - st.bsig[o]) + 4.0 * nb * kEps * fmax(st.btn[o], fabs(st.bsig[o])) + pivmin;
  for (int it = 0; it < 64; ++it) {
    if (lo > 0.0 && hi - lo <= 4.0 * kEps * hi) break;  // same on every lane
    double x;
    if (lo == 0.0) {
      x = ldexp(hi, lane - 64);
    } else if (hi > 1.5 * lo) {
      x = lo * exp2(log2(hi / lo) * (double)(lane + 1) / 65.0);
    } else {
      x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    }
    x = fmin(fmax(x, lo), hi);
    const int c = negcount(Ds, Ls, o, nb, x, pivmin);
    // counts rise with x: the first lane whose count passes `want` closes the bracket
    const uint64_t above = __ballot(c > want);
    const int b = above ? __ffsll((unsigned long long)above) - 1 : 64;
    const double nhi = b < 64 ? readlane_d(x, b) : hi;
    const double nlo = b > 0 ? readlane_d(x, b - 1) : lo;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) st.mu[g] = 0.5 * (lo + hi);
}

// Phases 4 and 5.
__global__ __launch_bounds__(kT) void syev_vectors_kernel(int n, double* d_out, double* W, double* scratch) {
  __shared__ double A[kMaxL * kS];  // the eigenvectors Z of T, then the reflectors
  __shared__ double d[kMaxL], tau[kMaxL], pw[kMaxL];
  __shared__ double Dr[kMaxL], Lr[kMaxL], LLD[kMaxL], mu[kMaxL], shift[kMaxL];
  __shared__ double bsig[kMaxL];
  __shared__ double red[kT / 64];
  __shared__ int bstart[kMaxL], bsize[kMaxL], cl0[kMaxL], incl[kMaxL], rank_s[kMaxL];
  __shared__ int gs_list[kMaxL], slot_s[kMaxL];
  __shared__ double lds_lp[kLdsSlots * kMaxL];
  __shared__ int sh_int[4];
  double* house = scratch;                   // kMaxL x kMaxL reflectors
  double* lwork = scratch + kMaxL * kMaxL;   // per-column L+ of the cluster solves
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const EigState st = eig_state(scratch);
  for (int j = tid; j < n; j += kT) {
    d[j] = st.d[j];
    tau[j] = st.tau[j];
    Dr[j] = st.Dr[j];
    Lr[j] = st.Lr[j];
    LLD[j] = st.LLD[j];
    mu[j] = st.mu[j];
    bsig[j] = st.bsig[j];
    bstart[j] = st.bstart[j];
    bsize[j] = st.bsize[j];
  }
  const double pivmin = st.misc[0];
  __syncthreads();

  // ---------------------------------------------------------------- 4. eigenvectors of T
  for (int idx = tid; idx < n * n; idx += kT) A[(idx / n) * kS + (idx % n)] = 0.0;
  if (tid < n) {
    const int g = tid, o = bstart[g], nb = bsize[g];
    int c = g;
    if (nb > 1)
      while (c > o && mu[c] - mu[c - 1] < kMinRelGap * mu[c]) --c;
    cl0[g] = c;
    const bool after = nb > 1 && g + 1 < o + nb && mu[g + 1] - mu[g] < kMinRelGap * mu[g + 1];
    incl[g] = (c < g) || after;
  }
  __syncthreads();
  if (tid < n) {
    const int g = tid, o = bstart[g], nb = bsize[g], last = o + nb - 1;
    double* z = A + g;  // column g: z[i * kS]
    if (nb == 1) {
      z[o * kS] = 1.0;
    } else {
      const double lam = mu[g];
      // stationary transform top-down: s_i into z
      double s = -lam;
#pragma unroll 8
      for (int i = o; i < last; ++i) {
        z[i * kS] = s;
        const double dp = guard(Dr[i] + s, pivmin);
        s = (Dr[i] * Lr[i] * rcp2(dp)) * Lr[i] * s - lam;
      }
      z[last * kS] = s;
      // progressive transform bottom-up: gamma_i = s_i + p_i + lam, U-_i into z
      double p = Dr[last] - lam;
      int r = last;
      double gbest = fabs(z[last * kS] + p + lam);
#pragma unroll 8
      for (int i = last - 1; i >= o; --i) {
        const double dm = guard(LLD[i] + p, pivmin);
        const double t = Dr[i] * rcp2(dm);
        const double um = Lr[i] * t;
        p = p * t - lam;
        const double gam = fabs(z[i * kS] + p + lam);
        z[i * kS] = um;
        if (gam < gbest) {
          gbest = gam;
          r = i;
        }
      }
      // L+_i above r, top-down again
      s = -lam;
#pragma unroll 8
      for (int i = o; i < r; ++i) {
        const double dp = guard(Dr[i] + s, pivmin);
        const double lp = Dr[i] * Lr[i] * rcp2(dp);
        z[i * kS] = lp;
        s = lp * Lr[i] * s - lam;
      }
      double u = (r < last) ? z[r * kS] : 0.0;
      z[r * kS] = 1.0;
      double zj = 1.0, nrm = 1.0;
#pragma unroll 8
      for (int i = r; i < last; ++i) {
        const double unext = (i + 1 < last) ? z[(i + 1) * kS] : 0.0;
        zj = -u * zj;
        z[(i + 1) * kS] = zj;
        nrm += zj * zj;
        u = unext;
      }
      zj = 1.0;
#pragma unroll 8
      for (int i = r - 1; i >= o; --i) {
        zj = -z[i * kS] * zj;
        z[i * kS] = zj;
        nrm += zj * zj;
      }
      const double inv = 1.0 / sqrt(nrm);
      if (incl[g]) {
        double nrm2 = 0.0;
        for (int i = o; i <= last; ++i) {
          const double v = z[i * kS] * inv + 1e-3 * jitter(g, i);
          z[i * kS] = v;
          nrm2 += v * v;
        }
        const double inv2 = 1.0 / sqrt(nrm2);
        for (int i = o; i <= last; ++i) z[i * kS] *= inv2;
      } else {
        for (int i = o; i <= last; ++i) z[i * kS] *= inv;
      }
    }
    // separated shifts for the cluster solves
    if (incl[g]) {
      double sh = mu[g];
      if (cl0[g] < g) {
        // walk the cluster from its first member (serial, once per member: cluster sizes are small)
        double prev = mu[cl0[g]];
        for (int t = cl0[g] + 1; t <= g; ++t) {
          prev = fmax(mu[t], prev + 10.0 * kEps * mu[t]);
        }
        sh = prev;
      }
      shift[g] = sh;
    }
  }
  if (tid == 0) {
    int any = 0, ngs = 0, nslot = 0;
    for (int g = 0; g < n; ++g) {
      any |= incl[g];
      slot_s[g] = incl[g] ? nslot++ : -1;
      if (incl[g] && cl0[g] < g) gs_list[ngs++] = g;
    }
    sh_int[1] = any;
    sh_int[2] = ngs;
  }
  __syncthreads();
  if (sh_int[1]) {
    const int ngs = sh_int[2];
    for (int it = 0; it < kClusterIters; ++it) {
      // (L D L^T - shift I) y = z for every clustered column, in place
      if (tid < n && incl[tid]) {
        const int g = tid, o = bstart[g], last = o + bsize[g] - 1;
        const double lam = shift[g];
        // pivots floored relative to the shift, so the solve keeps the representation's
        // relative accuracy (an absolute floor would mix in neighbouring eigenvectors)
        const double pfl = fmax(kEps * lam, pivmin);
        double* z = A + g;
        // L+ of this column's solve: LDS for the first clustered columns, else global scratch
        const int sl = slot_s[g];
        double* lp = (sl < kLdsSlots) ? lds_lp + sl * kMaxL : lwork + (size_t)g * kMaxL;
        double s = -lam, yprev = 0.0, lprev = 0.0;
#pragma unroll 8
        for (int i = o; i <= last; ++i) {
          const double dp = guard(Dr[i] + s, pfl);
          const double rp = rcp2(dp);
          const double y = z[i * kS] - lprev * yprev;
          yprev = y;
          z[i * kS] = y * rp;
          if (i < last) {
            lprev = Dr[i] * Lr[i] * rp;
            lp[i] = lprev;
            s = lprev * Lr[i] * s - lam;
          }
        }
        double ynext = z[last * kS], ymax = fabs(ynext), nrm = ynext * ynext;
        for (int i = last - 1; i >= o; i -= 8) {
          // the L+ values come from global memory: fetch eight before the dependent chain
          double lv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) lv[u] = (i - u >= o) ? lp[i - u] : 0.0;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (i - u >= o) {
              const double y = z[(i - u) * kS] - lv[u] * ynext;
              z[(i - u) * kS] = y;
              ynext = y;
              ymax = fmax(ymax, fabs(y));
              nrm += y * y;
            }
          }
        }
        if (nrm > 0.0 && nrm <= 1e300) {
          const double inv = 1.0 / sqrt(nrm);
#pragma unroll 8
          for (int i = o; i <= last; ++i) z[i * kS] *= inv;
        } else if (ymax > 0.0) {  // sum of squares out of range: scale by the largest entry first
          const double sc = 1.0 / ymax;
          double nrm2 = 0.0;
#pragma unroll 8
          for (int i = o; i <= last; ++i) {
            const double y = z[i * kS] * sc;
            z[i * kS] = y;
            nrm2 += y * y;
          }
          const double inv = 1.0 / sqrt(nrm2);
          for (int i = o; i <= last; ++i) z[i * kS] *= inv;
        }
      }
      __syncthreads();
      for (int gi = 0; gi < ngs; ++gi) {
        const int g = gs_list[gi], c0 = cl0[g];
        for (int pass = 0; pass < 2; ++pass) {
          for (int i = c0 + wave; i < g; i += kT / 64) {
            double s = 0.0;
            for (int r2 = lane; r2 < n; r2 += 64) s += A[r2 * kS + i] * A[r2 * kS + g];
            s = wave_sum(s);
            if (lane == 0) pw[i] = s;
          }
          __syncthreads();
          if (tid < n) {
            double v = A[tid * kS + g];
            for (int i = c0; i < g; ++i) v -= pw[i] * A[tid * kS + i];
            A[tid * kS + g] = v;
          }
          __syncthreads();
        }
        const double part = (tid < n) ? A[tid * kS + g] * A[tid * kS + g] : 0.0;
        const double nn = block_sum(part, red);
        if (tid < n && nn > 0.0) A[tid * kS + g] *= 1.0 / sqrt(nn);
        __syncthreads();
      }
    }
  }

  // ---------------------------------------------------------------- eigenvalues ascending
  if (tid < n) {
    const int g = tid, o = bstart[g];
    const double v = (bsize[g] > 1) ? mu[g] + bsig[o] : d[g];
    mu[g] = v;  // own slot only; read below after the barrier
  }
  __syncthreads();
  if (tid < n) {
    const double v = mu[tid];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double u2 = mu[j];
      r += (u2 < v) || (u2 == v && j < tid);
    }
    rank_s[tid] = r;
    d_out[r] = v;
  }

  // ---------------------------------------------------------------- 5. back-transformation
  // Z into registers: wave w < 8 owns columns 16w..16w+15; lane L holds columns
  // 16w + 2 (L/8) and the next one, rows L%8 + 8q (q = 0..15). The eight lanes of a column
  // pair read a reflector's entries from consecutive LDS words, and each entry read serves two
  // columns (half the LDS reads per reflector of one column per lane). The reflectors move
  // into the freed LDS matrix (row k holds v_k for rows k+1..n-1), and every wave applies all
  // of them to its own columns with no further barrier: s = v^T z summed over the eight lanes
  // of a column, z -= tau s v. Waves 8..15 have no columns here.
  const int zc = 16 * wave + 2 * (lane >> 3), zr0 = lane & 7;
  const bool zw = wave < 8;  // uniform per wave
  double z0[16], z1[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int row = zr0 + 8 * q;
    z0[q] = (zw && row < n && zc < n) ? A[row * kS + zc] : 0.0;
    z1[q] = (zw && row < n && zc + 1 < n) ? A[row * kS + zc + 1] : 0.0;
  }
  __syncthreads();
  if (n > 2) {  // uniform; with n <= 2 there are no reflectors
    // a thread's loads are issued eight at a time before their LDS writes (indices clamped
    // into the reflector block, so the loads need no branch), not one global round trip per
    // element; eight keep the registers of Z and the staged values within budget
    constexpr int kCopy = (kMaxL * kMaxL + kT - 1) / kT, kBatch = 8;
    const int total = (n - 2) * kMaxL;
#pragma unroll
    for (int u0 = 0; u0 < kCopy; u0 += kBatch) {
      double hv[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) hv[u] = house[min(tid + (u0 + u) * kT, total - 1)];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int idx = tid + (u0 + u) * kT;
        const int k = idx / kMaxL, i = idx - k * kMaxL;
        if (idx < total && i < n - k - 1) A[k * kS + i] = hv[u];
      }
    }
  }
  __syncthreads();
  if (zw) {
    for (int k = n - 3; k >= 0; --k) {
      const double tk = tau[k];
      if (tk == 0.0) continue;  // uniform
      const double* hv = A + k * kS;
      double vq[16];
      double sa[2] = {0.0, 0.0}, sb[2] = {0.0, 0.0};  // two partial sums per column
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int row = zr0 + 8 * q;
        vq[q] = (row >= k + 1 && row < n) ? hv[row - k - 1] : 0.0;
        sa[q & 1] += vq[q] * z0[q];
        sb[q & 1] += vq[q] * z1[q];
      }
      const double ta = tk * oct_allsum(sa[0] + sa[1]);
      const double tb = tk * oct_allsum(sb[0] + sb[1]);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        z0[q] -= ta * vq[q];
        z1[q] -= tb * vq[q];
      }
    }
    const int col0 = zc < n ? rank_s[zc] : 0, col1 = zc + 1 < n ? rank_s[zc + 1] : 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int row = zr0 + 8 * q;
      if (row < n) {
        if (zc < n) W[(size_t)row * n + col0] = z0[q];
        if (zc + 1 < n) W[(size_t)row * n + col1] = z1[q];
      }
    }
  }
}

}  // namespace

size_t eig_scratch_bytes() {
  return (2 * (size_t)kMaxL * kMaxL + kStateDoubles) * sizeof(double) + 2 * (size_t)kMaxL * sizeof(int);
}

void launch_eig(const double* G, int ldg, int l, double* d, double* W, double* scratch, hipStream_t st) {
  syev_tridiag_kernel<<<1, kT, 0, st>>>(G, ldg, l, scratch);
  syev_bisect_kernel<<<(unsigned)((l + kBisWaves - 1) / kBisWaves), 64 * kBisWaves, 0, st>>>(l, scratch);
  syev_vectors_kernel<<<1, kT, 0, st>>>(l, d, W, scratch);
}

}  // namespace frpca
