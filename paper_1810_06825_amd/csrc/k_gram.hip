// Gram matrix B = X^T X of a tall panel (Alg. 2 step 1), FP32 data, FP64 accumulation on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64). Products of FP32 values are exact in FP64,
// so the only rounding is the FP64 accumulation.
//
// Each MFMA multiplies a 16x4 tile of X^T by a 4x16 tile of X: lane l supplies
// X[r0 + l/16][16*I + l%16] as the A operand (tile row I) and the same formula with J as the
// B operand; the 16x16 result tile is held 4 values per lane: value q of lane l is row
// l/16 + 4q, column l%16 (layout checked on gfx950). The l x l output is covered by NT x NT tiles (NT = ceil(l/16) rounded to even);
// for the symmetric Gram only the NT(NT+1)/2 upper tiles are computed. The four waves of a
// block split the tiles and walk the same rows 4 at a time. Each block writes its partial
// tiles; a second kernel adds the partials of all blocks in block order (deterministic).
#include <type_traits>

#include "kernels.h"

namespace frpca {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kGramMaxBlocks = 512;
constexpr int kMaxPairs = 64;  // 8 x 8 tiles

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int pair_i(int nt, bool sym, int p) {
  if (!sym) return p / nt;
  int i = 0;
  while (p >= nt - i) {
    p -= nt - i;
    ++i;
  }
  return i;
}
constexpr int pair_j(int nt, bool sym, int p) {
  if (!sym) return p % nt;
  int i = 0;
  while (p >= nt - i) {
    p -= nt - i;
    ++i;
  }
  return i + p;
}
constexpr int npairs(int nt, bool sym) { return sym ? nt * (nt + 1) / 2 : nt * nt; }

template <int NT, bool SYM, int WAVE>
__device__ __forceinline__ void gram_wave(const float* X1, int ld1, const float* X2, int ld2, int64_t r0,
                                          int64_t r1, int l, double* out) {
  constexpr int NP = npairs(NT, SYM);
  constexpr int PPW = (NP - WAVE + 3) / 4;  // pairs p = WAVE + 4q
  const int lane = threadIdx.x & 63;
  const int kr = lane >> 4, cc = lane & 15;
  d4 acc[PPW > 0 ? PPW : 1];
#pragma unroll
  for (int q = 0; q < (PPW > 0 ? PPW : 1); ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0; r < r1; r += 4) {
    const int64_t rr = r + kr;
    const bool ok = rr < r1;
    double a[NT], b[NT];
#pragma unroll
    for (int I = 0; I < NT; ++I) {
      const int c = 16 * I + cc;
      a[I] = (ok && c < l) ? (double)X1[rr * ld1 + c] : 0.0;
      if constexpr (!SYM) b[I] = (ok && c < l) ? (double)X2[rr * ld2 + c] : 0.0;
    }
    static_for<0, PPW>([&](auto qc) {
      constexpr int p = WAVE + 4 * decltype(qc)::value;
      constexpr int I = pair_i(NT, SYM, p), J = pair_j(NT, SYM, p);
      if constexpr (SYM) acc[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], a[J], acc[qc], 0, 0, 0);
      else acc[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], b[J], acc[qc], 0, 0, 0);
    });
  }
  static_for<0, PPW>([&](auto qc) {
    constexpr int p = WAVE + 4 * decltype(qc)::value;
    double* o = out + (size_t)p * 256 + lane * 4;
    o[0] = acc[qc][0];
    o[1] = acc[qc][1];
    o[2] = acc[qc][2];
    o[3] = acc[qc][3];
  });
}

template <int NT, bool SYM>
__global__ __launch_bounds__(256) void gram_kernel(const float* X1, int ld1, const float* X2, int ld2,
                                                   int64_t rows, int l, int64_t rows_per_block, double* partial) {
  constexpr int NP = npairs(NT, SYM);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(rows, r0 + rows_per_block);
  double* out = partial + (size_t)blockIdx.x * NP * 256;
  switch (threadIdx.x >> 6) {
    case 0: gram_wave<NT, SYM, 0>(X1, ld1, X2, ld2, r0, r1, l, out); break;
    case 1: gram_wave<NT, SYM, 1>(X1, ld1, X2, ld2, r0, r1, l, out); break;
    case 2: gram_wave<NT, SYM, 2>(X1, ld1, X2, ld2, r0, r1, l, out); break;
    default: gram_wave<NT, SYM, 3>(X1, ld1, X2, ld2, r0, r1, l, out); break;
  }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* partial, int nblk, int nt, bool sym,
                                                          int l, double* G, int ldg) {
  const int np = sym ? nt * (nt + 1) / 2 : nt * nt;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= np * 256) return;
  const int p = idx >> 8, t = idx & 255, lane = t >> 2, r = t & 3;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[((size_t)b * np + p) * 256 + t];
  int I, J;
  if (sym) {
    int q = p;
    I = 0;
    while (q >= nt - I) {
      q -= nt - I;
      ++I;
    }
    J = I + q;
  } else {
    I = p / nt;
    J = p % nt;
  }
  const int i = 16 * I + (lane >> 4) + 4 * r;
  const int j = 16 * J + (lane & 15);
  if (i >= l || j >= l) return;
  if (sym) {
    if (I == J && i > j) return;
    G[(size_t)i * ldg + j] = s;
    G[(size_t)j * ldg + i] = s;
  } else {
    G[(size_t)i * ldg + j] = s;
  }
}

template <bool SYM>
void gram_dispatch(int nt, unsigned grid, const float* X1, int ld1, const float* X2, int ld2, int64_t rows, int l,
                   int64_t rpb, double* partial, hipStream_t st) {
  switch (nt) {
    case 2: gram_kernel<2, SYM><<<grid, 256, 0, st>>>(X1, ld1, X2, ld2, rows, l, rpb, partial); break;
    case 4: gram_kernel<4, SYM><<<grid, 256, 0, st>>>(X1, ld1, X2, ld2, rows, l, rpb, partial); break;
    case 6: gram_kernel<6, SYM><<<grid, 256, 0, st>>>(X1, ld1, X2, ld2, rows, l, rpb, partial); break;
    default: gram_kernel<8, SYM><<<grid, 256, 0, st>>>(X1, ld1, X2, ld2, rows, l, rpb, partial); break;
  }
}

}  // namespace

size_t gram_partial_bytes(int /*l*/) { return (size_t)kGramMaxBlocks * kMaxPairs * 256 * sizeof(double); }

void launch_gram(const void* X1, bool /*bf16*/, int ld1, const float* X2, int ld2, int64_t rows, int l,
                 double* partial, double* G, int ldg, hipStream_t st) {
  int nt = (l + 15) / 16;
  nt += nt & 1;
  const bool sym = (X2 == nullptr);
  int64_t grid = (rows + 63) / 64;
  if (grid > kGramMaxBlocks) grid = kGramMaxBlocks;
  if (grid < 1) grid = 1;
  int64_t rpb = (rows + grid - 1) / grid;
  rpb = (rpb + 3) / 4 * 4;
  const float* x1 = static_cast<const float*>(X1);
  if (sym) gram_dispatch<true>(nt, (unsigned)grid, x1, ld1, x1, ld1, rows, l, rpb, partial, st);
  else gram_dispatch<false>(nt, (unsigned)grid, x1, ld1, X2, ld2, rows, l, rpb, partial, st);
  const int np = sym ? nt * (nt + 1) / 2 : nt * nt;
  gram_reduce_kernel<<<(unsigned)((np * 256 + 255) / 256), 256, 0, st>>>(partial, (int)grid, nt, sym, l, G, ldg);
}

}  // namespace frpca
