// Adjoint of the truncated SVD projected on the sparsity pattern (the differentiated form).
//
// With J = U^T dU, K = V^T dV, F_ij = 1/(s_j^2 - s_i^2) (i != j; 0 when the gap is <= 1e-12
// s_1^2) and S+ = diag(1/s or 0), the gradient
//   dA = U M V^T + (dU - U J) S+ V^T + U S+ (dV - V K)^T,
//   M  = (F o (J - J^T)) S + diag(dS) + S (F o (K - K^T)),
// is regrouped as dA = L1 V^T + U R2^T with L1 = U (M - J S+) + dU S+ and R2 = (dV - V K) S+,
// so only its values at the stored nonzeros are formed: dval[e] = L1[r].V[c] + U[r].R2[c]
// (sampled dense-dense product, SDDMM), minus a per-column term corr[c] for the centred
// matrix (k_center.hip). The k x k algebra runs in FP64 in one workgroup.
#include "kernels.h"

namespace frpca {
namespace {

__global__ __launch_bounds__(256) void adjoint_small_kernel(const double* J, const double* K, const float* S,
                                                            const float* dS, int k, int has_du, int has_dv,
                                                            double* CU, double* CV, double* SP) {
  const double s1 = (double)S[0];
  const double gap_tol = 1e-12 * s1 * s1;
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    const int i = idx / k, j = idx - i * k;
    const double si = (double)S[i], sj = (double)S[j];
    const double spj = sj > 0.0 ? 1.0 / sj : 0.0;
    double F = 0.0;
    if (i != j) {
      const double d = sj * sj - si * si;
      if (fabs(d) > gap_tol) F = 1.0 / d;
    }
    double m = 0.0;
    double jij = 0.0;
    if (has_du) {
      jij = J[idx];
      m += F * (jij - J[j * k + i]) * sj;
    }
    if (has_dv) m += si * F * (K[idx] - K[j * k + i]);
    if (i == j && dS) m += (double)dS[i];
    CU[idx] = m - jij * spj;
    CV[idx] = has_dv ? -K[idx] * spj : 0.0;
    SP[idx] = (i == j) ? spj : 0.0;
  }
}

// One wave per row: lanes hold two columns of P1[r] / P2[r], gather Q1[c] / Q2[c] per
// nonzero and reduce across the wave in a fixed butterfly order.
__global__ __launch_bounds__(256) void sddmm_kernel(const int32_t* rp, const int32_t* col, int64_t m, int w,
                                                    const float* P1, const float* Q1, const float* P2,
                                                    const float* Q2, const float* corr, float* dval) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wstride = (int64_t)gridDim.x * 4;
  const int c0 = 2 * lane, c1 = 2 * lane + 1;
  const bool a0 = c0 < w, a1 = c1 < w;
  for (int64_t r = wave0; r < m; r += wstride) {
    const float* p1 = P1 + (size_t)r * w;
    const float x0 = a0 ? p1[c0] : 0.f, x1 = a1 ? p1[c1] : 0.f;
    float y0 = 0.f, y1 = 0.f;
    if (P2) {
      const float* p2 = P2 + (size_t)r * w;
      y0 = a0 ? p2[c0] : 0.f;
      y1 = a1 ? p2[c1] : 0.f;
    }
    const int e0 = rp[r], e1 = rp[r + 1];
    for (int e = e0; e < e1; ++e) {
      const int c = col[e];
      const float* q1 = Q1 + (size_t)c * w;
      float part = (a0 ? x0 * q1[c0] : 0.f) + (a1 ? x1 * q1[c1] : 0.f);
      if (Q2) {
        const float* q2 = Q2 + (size_t)c * w;
        part += (a0 ? y0 * q2[c0] : 0.f) + (a1 ? y1 * q2[c1] : 0.f);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
      if (lane == 0) dval[e] = corr ? part - corr[c] : part;
    }
  }
}

// Paired form (k a multiple of 4, rows 16-byte aligned): lanes 0-31 take the even nonzero of
// each pair of a row, lanes 32-63 the odd one, a lane covering four columns; the column
// indices come 64 at a time in one coalesced load and reach the pairs by readlane; eight pairs
// are gathered before any is reduced, and each half-wave sum runs on DPP row shifts (lanes 31
// and 63 end with the totals), so no LDS shuffles are needed.
constexpr int kSdPairs = 8;
#ifndef FRPCA_SDDMM_QUAD
#define FRPCA_SDDMM_QUAD 1
#endif

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dppf(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, true));
}

// Sum over each half-wave, valid in lanes 31 and 63 (row shifts 1, 2, 4, 8 then the row-15
// broadcast into rows 1 and 3; out-of-row sources read 0).
__device__ __forceinline__ float half_sum_last(float v) {
  v += dppf<0x111, 0xF>(v);
  v += dppf<0x112, 0xF>(v);
  v += dppf<0x114, 0xF>(v);
  v += dppf<0x118, 0xF>(v);
  v += dppf<0x142, 0xA>(v);
  return v;
}

// Sum over each row of 16 lanes, valid in its lane 15.
__device__ __forceinline__ float row_sum_last(float v) {
  v += dppf<0x111, 0xF>(v);
  v += dppf<0x112, 0xF>(v);
  v += dppf<0x114, 0xF>(v);
  v += dppf<0x118, 0xF>(v);
  return v;
}

// TWO: the second product term is present; CORR: the per-column centring term is present. Both
// are compile-time so the kSdPairs gathers of a batch issue back to back before any arithmetic
// (a run-time test between them makes the compiler wait for each gather in turn). G: nonzeros
// per gather instruction, 2 (half-waves of 32 lanes, panels up to 128 columns) or 4 (rows of
// 16 lanes, panels up to 64 columns, whose pairs would leave half of each half-wave idle).
template <bool TWO, bool CORR, int G>
__global__ __launch_bounds__(256) void sddmm4_kernel(const int32_t* rp, const int32_t* col, int64_t m, int w,
                                                     const float* P1, const float* Q1, const float* P2,
                                                     const float* Q2, const float* corr, float* dval) {
  static_assert(G == 2 || G == 4, "two or four nonzeros per gather");
  constexpr int kLanes = 64 / G;  // lanes per nonzero
  const int lane = threadIdx.x & 63, half = lane / kLanes;
  const int c4 = 4 * (lane % kLanes);
  const bool act = c4 < w;
  const int gc = act ? c4 : 0;
  const int64_t wave0 = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wstride = (int64_t)gridDim.x * 4;
  int64_t r = wave0;
  if (r >= m) return;
  // The metadata of a row (its panel entries x, y and its first 64 column indices) is loaded
  // one row ahead and its extent two rows ahead, so a row's first gathers do not wait for the
  // row pointer and then the column indices in turn. Inactive lanes read column 0 of a panel
  // row (in bounds); their products are dropped below.
  auto load_x = [&](int64_t row, float4& xo, float4& yo) {
    xo = *reinterpret_cast<const float4*>(P1 + (size_t)row * w + gc);
    yo = make_float4(0.f, 0.f, 0.f, 0.f);
    if (TWO) yo = *reinterpret_cast<const float4*>(P2 + (size_t)row * w + gc);
  };
  int e0 = rp[r], e1 = rp[r + 1];
  float4 x, y;
  load_x(r, x, y);
  int cidx = e0 + lane < e1 ? col[e0 + lane] : 0;
  int64_t rn = r + wstride;
  int e0n = 0, e1n = 0;
  if (rn < m) {
    e0n = rp[rn];
    e1n = rp[rn + 1];
  }
  for (;;) {
    float4 xn = x, yn = y;
    int cidxn = 0, e0nn = 0, e1nn = 0;
    const int64_t rnn = rn + wstride;
    if (rn < m) {
      load_x(rn, xn, yn);
      cidxn = e0n + lane < e1n ? col[e0n + lane] : 0;
      if (rnn < m) {
        e0nn = rp[rnn];
        e1nn = rp[rnn + 1];
      }
    }
    // one chunk of up to 64 nonzeros whose column indices the lanes hold in ci; past the row end
    // the index is 0, a valid column whose result is discarded
    auto chunk = [&](int ec, int ci) {
      const int nb = __builtin_amdgcn_readfirstlane(min(64, e1 - ec));
      for (int b = 0; b < nb; b += G * kSdPairs) {
        const int e = ec + b;
        int cs[kSdPairs];
        float4 q[kSdPairs], q2[kSdPairs];
        float cv[kSdPairs];
#pragma unroll
        for (int p = 0; p < kSdPairs; ++p) {
          const int ce = __builtin_amdgcn_readlane(ci, (b + G * p) & 63);
          const int co = __builtin_amdgcn_readlane(ci, (b + G * p + 1) & 63);
          if constexpr (G == 2) {
            cs[p] = half ? co : ce;
          } else {
            const int c2 = __builtin_amdgcn_readlane(ci, (b + G * p + 2) & 63);
            const int c3 = __builtin_amdgcn_readlane(ci, (b + G * p + 3) & 63);
            cs[p] = half == 0 ? ce : half == 1 ? co : half == 2 ? c2 : c3;
          }
          q[p] = q2[p] = make_float4(0.f, 0.f, 0.f, 0.f);
          cv[p] = 0.f;
          // groups past the chunk's end are not gathered (the test is uniform over the wave)
          if (b + G * p < nb) {
            q[p] = *reinterpret_cast<const float4*>(Q1 + (size_t)cs[p] * w + gc);
            if (TWO) q2[p] = *reinterpret_cast<const float4*>(Q2 + (size_t)cs[p] * w + gc);
            if (CORR) cv[p] = corr[cs[p]];
          }
        }
#pragma unroll
        for (int p = 0; p < kSdPairs; ++p) {
          float s = x.x * q[p].x + x.y * q[p].y + x.z * q[p].z + x.w * q[p].w;
          if (TWO) s += y.x * q2[p].x + y.y * q2[p].y + y.z * q2[p].z + y.w * q2[p].w;
          const float t = G == 2 ? half_sum_last(act ? s : 0.f) : row_sum_last(act ? s : 0.f);
          const int ee = e + G * p + half;
          if (lane % kLanes == kLanes - 1 && ee < e1) dval[ee] = CORR ? t - cv[p] : t;
        }
      }
    };
    // The first chunk is a code path of its own: its indices arrived with the previous row, so
    // its gathers issue without waiting for the loads just issued for the next row.
    if (e0 < e1) chunk(e0, cidx);
    for (int ec = e0 + 64; ec < e1; ec += 64) chunk(ec, ec + lane < e1 ? col[ec + lane] : 0);
    if (rn >= m) break;
    r = rn;
    rn = rnn;
    x = xn;
    y = yn;
    cidx = cidxn;
    e0 = e0n;
    e1 = e1n;
    e0n = e0nn;
    e1n = e1nn;
  }
}

}  // namespace

void launch_adjoint_small(const double* J, const double* K, const float* S, const float* dS, int k, bool has_du,
                          bool has_dv, double* CU, double* CV, double* SP, hipStream_t st) {
  adjoint_small_kernel<<<1, 256, 0, st>>>(J, K, S, dS, k, has_du ? 1 : 0, has_dv ? 1 : 0, CU, CV, SP);
}

void launch_sddmm(const int32_t* rp, const int32_t* col, int64_t m, int w, const float* P1, const float* Q1,
                  const float* P2, const float* Q2, float* dval, hipStream_t st, const float* corr) {
  if (m <= 0) return;
  int64_t grid = (m + 3) / 4;
  if (grid > 65536) grid = 65536;
  auto al = [](const float* p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) % 16) == 0; };
  if (w % 4 == 0 && w <= 128 && al(P1) && al(Q1) && al(P2) && al(Q2)) {
    const bool two = P2 != nullptr && Q2 != nullptr;
    auto go = [&](auto g) {
      constexpr int G = decltype(g)::value;
      if (two && corr) sddmm4_kernel<true, true, G><<<(unsigned)grid, 256, 0, st>>>(rp, col, m, w, P1, Q1, P2, Q2, corr, dval);
      else if (two) sddmm4_kernel<true, false, G><<<(unsigned)grid, 256, 0, st>>>(rp, col, m, w, P1, Q1, P2, Q2, corr, dval);
      else if (corr) sddmm4_kernel<false, true, G><<<(unsigned)grid, 256, 0, st>>>(rp, col, m, w, P1, Q1, P2, Q2, corr, dval);
      else sddmm4_kernel<false, false, G><<<(unsigned)grid, 256, 0, st>>>(rp, col, m, w, P1, Q1, P2, Q2, corr, dval);
    };
    if (w <= 64 && FRPCA_SDDMM_QUAD) go(std::integral_constant<int, 4>{});
    else go(std::integral_constant<int, 2>{});
    return;
  }
  sddmm_kernel<<<(unsigned)grid, 256, 0, st>>>(rp, col, m, w, P1, Q1, P2, Q2, corr, dval);
}

}  // namespace frpca
