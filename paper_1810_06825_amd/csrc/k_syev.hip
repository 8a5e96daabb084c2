// Symmetric eigendecomposition of the l x l Gram matrix (Alg. 2 step 2), FP64, one workgroup
// of 16 waves. Householder tridiagonalization, then eigenpairs of the tridiagonal T by the
// multiple relatively robust representations idea (Dhillon & Parlett, 2004), then the
// back-transformation:
//
//  1. Q^T G Q = T by Householder reflectors H_k = I - tau_k v_k v_k^T, v_k(0) = 1 (Golub &
//     Van Loan, Alg. 8.3.1). G lives in LDS; step k needs three barriers: v_k (with the norm
//     of the next column reduced during the previous update), p = tau A22 v with p.v, and
//     the rank-2 update A22 -= v w^T + w v^T, w = p - (tau p.v / 2) v. The v_k go to a global
//     scratch buffer for step 5.
//  2. T splits where |e_j| <= eps ||T||. Each unreduced block gets a root representation
//     L D L^T = T - sigma I with every D_i > 0. For a Gram matrix sigma = -nb eps ||T_b||
//     works; otherwise sigma is the smallest eigenvalue (multisection on Sturm counts of T)
//     minus a margin that grows until D > 0. A positive definite L D L^T determines its
//     eigenvalues to high relative accuracy, so eigenvectors of eigenvalues with a relative
//     gap of 1e-3 or more come out numerically orthogonal without any reorthogonalization.
//  3. Eigenvalues mu of L D L^T by multisection on negative-pivot counts of the stationary
//     qd transform L D L^T - x I = L+ D+ L+^T (eight threads per eigenvalue, nine
//     subintervals per step, geometric points while the bracket spans a wide ratio), to a
//     relative width of 4 eps.
//  4. Each isolated eigenvector from the twisted factorization of L D L^T - mu I at the index
//     r where |gamma_r| = |s_r + p_r + mu| is smallest (stationary and progressive qd
//     transforms): z_r = 1, z_i = -L+_i z_i+1 above r, z_i+1 = -U-_i z_i below r. Eigenvalues
//     with a relative gap under 1e-3 form clusters; their vectors start from the twisted
//     ones (slightly perturbed) and take four steps of inverse iteration with shifts kept
//     10 eps apart, each followed by Gram-Schmidt (twice) against the earlier members.
//  5. W = H_0 H_1 ... H_{n-3} Z, eigenvalues sorted ascending (the order Alg. 2 and the final
//     selection ind = k+s:-1:s+1 rely on; ties in index order).
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kT = 1024;             // threads
constexpr int kS = kMaxL + 1;        // odd LDS row stride (doubles)
constexpr double kEps = 2.220446049250313e-16;
constexpr double kMinRelGap = 1e-3;  // relative gap below which eigenvalues form a cluster
constexpr int kClusterIters = 4;

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
// stationary qd transform.
__device__ int negcount(const double* D, const double* LLD, int o, int nb, double x, double pivmin) {
  double s = -x;
  int c = 0;
  for (int i = o; i < o + nb - 1; ++i) {
    const double dp = guard(D[i] + s, pivmin);
    c += dp < 0.0;
    s = (s / dp) * LLD[i] - x;
  }
  c += guard(D[o + nb - 1] + s, pivmin) < 0.0;
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

__global__ __launch_bounds__(kT) void syev_kernel(const double* G, int ldg, int n, double* d_out, double* W,
                                                  double* scratch) {
  __shared__ double A[kMaxL * kS];  // G, then the eigenvectors Z of T
  __shared__ double d[kMaxL], e[kMaxL], e2[kMaxL], tau[kMaxL], vk[kMaxL], pw[kMaxL];
  __shared__ double Dr[kMaxL], Lr[kMaxL], LLD[kMaxL], mu[kMaxL], shift[kMaxL];
  __shared__ double bsig[kMaxL], bgl[kMaxL], bgu[kMaxL], btn[kMaxL];
  __shared__ double red[kT / 64], red2[kT / 64];
  __shared__ int bstart[kMaxL], bsize[kMaxL], bbad[kMaxL], cl0[kMaxL], incl[kMaxL], rank_s[kMaxL];
  __shared__ int sh_int[4];
  __shared__ double sh_dbl[4];
  double* house = scratch;                   // kMaxL x kMaxL reflectors
  double* lwork = scratch + kMaxL * kMaxL;   // per-column L+ of the cluster solves
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row8 = tid >> 3, sub8 = tid & 7;

  for (int idx = tid; idx < n * n; idx += kT) {
    const int i = idx / n, j = idx - i * n;
    A[i * kS + j] = G[(size_t)i * ldg + j];
  }
  __syncthreads();

  // ---------------------------------------------------------------- 1. tridiagonalization
  {
    double part = 0.0;
    for (int i = 2 + tid; i < n; i += kT) part += A[i * kS] * A[i * kS];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double sigma = 0.0;
#pragma unroll
    for (int w = 0; w < kT / 64; ++w) sigma += red[w];
    const double x0 = A[(k + 1) * kS + k];
    double tk = 0.0, beta = x0, scal = 0.0;
    if (sigma != 0.0) {
      const double mu0 = sqrt(x0 * x0 + sigma);
      beta = (x0 <= 0.0) ? mu0 : -mu0;
      tk = (beta - x0) / beta;
      scal = 1.0 / (x0 - beta);
    }
    for (int i = tid; i < m; i += kT) {
      const double v = (i == 0) ? 1.0 : A[(k + 1 + i) * kS + k] * scal;
      vk[i] = v;
      house[(size_t)k * kMaxL + i] = v;
    }
    if (tid == 0) {
      tau[k] = tk;
      e[k] = beta;
      d[k] = A[k * kS + k];
    }
    __syncthreads();  // (1)
    double acc = 0.0;
    if (row8 < m) {
      const double* ar = A + (k + 1 + row8) * kS + (k + 1);
      for (int j = sub8; j < m; j += 8) acc += ar[j] * vk[j];
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    const double pr = tk * acc;
    if (row8 < m && sub8 == 0) pw[row8] = pr;
    double pv = (row8 < m && sub8 == 0) ? pr * vk[row8] : 0.0;
    pv = wave_sum(pv);
    if (lane == 0) red2[wave] = pv;
    __syncthreads();  // (2)
    double K = 0.0;
#pragma unroll
    for (int w = 0; w < kT / 64; ++w) K += red2[w];
    K *= 0.5 * tk;
    double part = 0.0;
    if (row8 < m) {
      const double vi = vk[row8], wi = pr - K * vi;
      double* ar = A + (k + 1 + row8) * kS + (k + 1);
      for (int j = sub8; j < m; j += 8) {
        const double vj = vk[j];
        const double a = ar[j] - (vi * (pw[j] - K * vj) + wi * vj);
        ar[j] = a;
        if (j == 0 && row8 >= 2) part += a * a;
      }
    }
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();  // (3)
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = A[(n - 2) * kS + (n - 2)];
      e[n - 2] = A[(n - 1) * kS + (n - 2)];
    }
    d[n - 1] = A[(n - 1) * kS + (n - 1)];
    e[n - 1] = 0.0;
  }
  __syncthreads();

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

  // ---------------------------------------------------------------- 3. eigenvalues of L D L^T
  {
    const int g = row8;
    const bool act = g < n && bsize[g] > 1;
    int o = 0, nb = 1, want = 0;
    double lo = 0.0, hi = 0.0;
    if (act) {
      o = bstart[g];
      nb = bsize[g];
      want = g - o;
      hi = (bgu[o] - bsig[o]) + 4.0 * nb * kEps * fmax(btn[o], fabs(bsig[o])) + pivmin;
    }
    for (int it = 0; it < 64; ++it) {
      const bool busy = act && !(lo > 0.0 && hi - lo <= 4.0 * kEps * hi);
      if (!__any(busy)) break;  // per wave; the eight lanes of a group agree on busy
      double x;
      if (lo == 0.0) {
        x = ldexp(hi, -7 * (8 - sub8));
      } else if (hi > 1.5 * lo) {
        x = lo * exp2(log2(hi / lo) * (double)(sub8 + 1) / 9.0);
      } else {
        x = lo + (hi - lo) * (double)(sub8 + 1) / 9.0;
      }
      x = fmin(fmax(x, lo), hi);
      const int c = busy ? negcount(Dr, LLD, o, nb, x, pivmin) : 0;
      int b = 8;
      double xb = hi, xb1 = lo;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int cs = __shfl(c, (lane & ~7) + s);
        const double xs = __shfl(x, (lane & ~7) + s);
        if (b == 8 && cs > want) {
          b = s;
          xb = xs;
        }
        if (b == 8) xb1 = xs;
      }
      if (busy) {
        lo = xb1;
        hi = xb;
      }
    }
    if (sub8 == 0 && g < n) mu[g] = act ? 0.5 * (lo + hi) : 0.0;
  }
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
      for (int i = o; i < last; ++i) {
        z[i * kS] = s;
        const double dp = guard(Dr[i] + s, pivmin);
        s = (Dr[i] * Lr[i] / dp) * Lr[i] * s - lam;
      }
      z[last * kS] = s;
      // progressive transform bottom-up: gamma_i = s_i + p_i + lam, U-_i into z
      double p = Dr[last] - lam;
      int r = last;
      double gbest = fabs(z[last * kS] + p + lam);
      for (int i = last - 1; i >= o; --i) {
        const double dm = guard(LLD[i] + p, pivmin);
        const double t = Dr[i] / dm;
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
      for (int i = o; i < r; ++i) {
        const double dp = guard(Dr[i] + s, pivmin);
        const double lp = Dr[i] * Lr[i] / dp;
        z[i * kS] = lp;
        s = lp * Lr[i] * s - lam;
      }
      double u = (r < last) ? z[r * kS] : 0.0;
      z[r * kS] = 1.0;
      double zj = 1.0, nrm = 1.0;
      for (int i = r; i < last; ++i) {
        const double unext = (i + 1 < last) ? z[(i + 1) * kS] : 0.0;
        zj = -u * zj;
        z[(i + 1) * kS] = zj;
        nrm += zj * zj;
        u = unext;
      }
      zj = 1.0;
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
    int any = 0;
    for (int g = 0; g < n; ++g) any |= incl[g];
    sh_int[1] = any;
  }
  __syncthreads();
  if (sh_int[1]) {
    for (int it = 0; it < kClusterIters; ++it) {
      // (L D L^T - shift I) y = z for every clustered column, in place
      if (tid < n && incl[tid]) {
        const int g = tid, o = bstart[g], last = o + bsize[g] - 1;
        const double lam = shift[g];
        // pivots floored relative to the shift, so the solve keeps the representation's
        // relative accuracy (an absolute floor would mix in neighbouring eigenvectors)
        const double pfl = fmax(kEps * lam, pivmin);
        double* z = A + g;
        double* lp = lwork + (size_t)g * kMaxL;
        double s = -lam, yprev = 0.0;
        for (int i = o; i <= last; ++i) {
          const double dp = guard(Dr[i] + s, pfl);
          const double y = z[i * kS] - ((i > o) ? lp[i - 1] * yprev : 0.0);
          yprev = y;
          z[i * kS] = y / dp;
          if (i < last) {
            const double l = Dr[i] * Lr[i] / dp;
            lp[i] = l;
            s = l * Lr[i] * s - lam;
          }
        }
        double ynext = z[last * kS], ymax = fabs(ynext);
        for (int i = last - 1; i >= o; --i) {
          const double y = z[i * kS] - lp[i] * ynext;
          z[i * kS] = y;
          ynext = y;
          ymax = fmax(ymax, fabs(y));
        }
        if (ymax > 0.0) {  // scale first: the solve output can be far from 1 in magnitude
          const double sc = 1.0 / ymax;
          double nrm = 0.0;
          for (int i = o; i <= last; ++i) {
            const double y = z[i * kS] * sc;
            z[i * kS] = y;
            nrm += y * y;
          }
          const double inv = 1.0 / sqrt(nrm);
          for (int i = o; i <= last; ++i) z[i * kS] *= inv;
        }
      }
      __syncthreads();
      for (int g = 0; g < n; ++g) {
        const int c0 = cl0[g];
        if (!incl[g] || c0 == g) continue;  // uniform
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

  // ---------------------------------------------------------------- 5. back-transformation
  for (int k = n - 3; k >= 0; --k) {
    const int m = n - k - 1;
    for (int i = tid; i < m; i += kT) vk[i] = house[(size_t)k * kMaxL + i];
    __syncthreads();
    const double tk = tau[k];
    double s = 0.0;
    if (row8 < n && tk != 0.0)
      for (int i = sub8; i < m; i += 8) s += vk[i] * A[(k + 1 + i) * kS + row8];
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    if (row8 < n && tk != 0.0) {
      const double ts = tk * s;
      for (int i = sub8; i < m; i += 8) A[(k + 1 + i) * kS + row8] -= ts * vk[i];
    }
    __syncthreads();
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
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += kT) {
    const int i = idx / n, g = idx - i * n;
    W[(size_t)i * n + rank_s[g]] = A[i * kS + g];
  }
}

}  // namespace

size_t eig_scratch_bytes() { return 2 * (size_t)kMaxL * kMaxL * sizeof(double); }

void launch_eig(const double* G, int ldg, int l, double* d, double* W, double* scratch, hipStream_t st) {
  syev_kernel<<<1, kT, 0, st>>>(G, ldg, l, d, W, scratch);
}

}  // namespace frpca
