// Gram matrix B = X^T X of a tall panel (Alg. 2 step 1), FP32 data, FP64 accumulation on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64). Products of FP32 values are exact in FP64,
// so the only rounding is the FP64 accumulation.
//
// Each MFMA multiplies a 16x4 tile of X^T by a 4x16 tile of X: lane l supplies
// X[r0 + l/16][16*I + l%16] as the A operand (tile row I) and the same formula with J as the
// B operand; the 16x16 result tile is held 4 values per lane: value q of lane l is row
// l/16 + 4q, column l%16 (layout checked on gfx950). The l x l output is covered by NT x NT tiles
// (NT = ceil(l/16), with 1 and 5 rounded up to 2 and 6);
// for the symmetric Gram only the NT(NT+1)/2 upper tiles are computed. The four waves of a
// block split the tiles and walk the same rows 4 at a time. On panels padded to 16 NT columns
// each wave keeps three row steps in flight in a ring of registers (unconditional loads, so the
// compiler waits for each buffer's own loads); the row loads, not the matrix cores, bound the
// one-step form. Each block writes its partial tiles; a second kernel adds the partials of all
// blocks in block order (deterministic).
#include <type_traits>

#include "kernels.h"

namespace frpca {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// FP32 variant (F32, symmetric Gram only): v_mfma_f32_16x16x4f32 on the FP32 inputs, whose
// partial sums over kFlushSteps row steps (16 rows per stream) are added into FP64 accumulators. Its 16 x 16
// result holds value q of lane l at row 4 (l/16) + q (the FP64 instruction: row l/16 + 4q);
// the partial tiles keep the layout of the instruction that made them and the reduction maps
// each back.
constexpr int kFlushSteps = 4;

constexpr int kGramThreads = 512;  // 8 waves: 4 groups of tile pairs x 2 interleaved row streams
constexpr int kGramMaxBlocks = 512;
constexpr int kMaxPairs = 64;      // 8 x 8 tiles
constexpr int kRedPart = 16;       // block-sum interleave of the reduction
constexpr int kRedEnt = 256 / kRedPart;  // entries per reduction workgroup

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

// Column order inside the tiles: groups of four tiles cover 64 consecutive columns (entry t of
// tile I is column 64 (I/4) + 4t + I%4), a trailing pair covers the next 32 (entry t of tile I
// is 64 G4 + 2t + (I - 4 G4)) and a last single tile the 16 after those (entry t is
// 64 G4 + 32 + t). A lane's operands for all tiles come from one 16-, 8- or 4-byte load per
// group. The reduction maps the tiles back.
__host__ __device__ constexpr int gram_col(int nt, int I, int t) {
  return (I < 4 * (nt / 4))       ? 64 * (I / 4) + 4 * t + (I % 4)
         : (I < 4 * (nt / 4) + 2) ? 64 * (nt / 4) + 2 * t + (I - 4 * (nt / 4))
                                  : 64 * (nt / 4) + 32 + t;
}

template <int NT>
__device__ __forceinline__ void gram_load(const float* X, int ld, int64_t row, bool ok, int l, int cc, bool vec,
                                          float v[NT]) {
  constexpr int G4 = NT / 4;
#pragma unroll
  for (int g = 0; g < G4; ++g) {
    const int c0 = 64 * g + 4 * cc;
    if (ok && vec && c0 + 3 < l) {
      const float4 w = *reinterpret_cast<const float4*>(X + (size_t)row * ld + c0);
      v[4 * g] = w.x;
      v[4 * g + 1] = w.y;
      v[4 * g + 2] = w.z;
      v[4 * g + 3] = w.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) v[4 * g + q] = (ok && c0 + q < l) ? X[(size_t)row * ld + c0 + q] : 0.f;
    }
  }
  if constexpr (NT % 4 == 3) {
    const int c1 = 64 * G4 + 32 + cc;
    v[4 * G4 + 2] = (ok && c1 < l) ? X[(size_t)row * ld + c1] : 0.f;
  }
  if constexpr (NT % 4 >= 2) {
    const int c0 = 64 * G4 + 2 * cc;
    if (ok && vec && c0 + 1 < l) {
      const float2 w = *reinterpret_cast<const float2*>(X + (size_t)row * ld + c0);
      v[4 * G4] = w.x;
      v[4 * G4 + 1] = w.y;
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) v[4 * G4 + q] = (ok && c0 + q < l) ? X[(size_t)row * ld + c0 + q] : 0.f;
    }
  }
}

#ifndef FRPCA_GRAM_RING
#define FRPCA_GRAM_RING 3
#endif
constexpr int kGramRing = FRPCA_GRAM_RING;  // row buffers per wave on the padded-panel path (0: off)

// Unconditional load of one row (16-byte aligned rows) whose 16 NT tile columns lie inside the
// panel: either ld >= 16 NT, or 2 ld >= 16 NT and the row is not the panel's last (the columns
// past ld are then the next row's first ones). Rows past r1 read row r1 - 1 (such loads only fill
// the pipeline past the last step and are never used). Columns past l come from the padding or
// the next row: a column only enters the Gram entries of its own row and column, which the
// reduction drops.
template <int NT>
__device__ __forceinline__ void gram_load_wide(const float* X, int ld, int64_t row, int64_t r1, int cc,
                                               float v[NT]) {
  constexpr int G4 = NT / 4;
  const float* p = X + (size_t)(row < r1 ? row : r1 - 1) * ld;
#pragma unroll
  for (int g = 0; g < G4; ++g) {
    const float4 w = *reinterpret_cast<const float4*>(p + 64 * g + 4 * cc);
    v[4 * g] = w.x;
    v[4 * g + 1] = w.y;
    v[4 * g + 2] = w.z;
    v[4 * g + 3] = w.w;
  }
  if constexpr (NT % 4 >= 2) {
    const float2 w = *reinterpret_cast<const float2*>(p + 64 * G4 + 2 * cc);
    v[4 * G4] = w.x;
    v[4 * G4 + 1] = w.y;
  }
  if constexpr (NT % 4 == 3) v[4 * G4 + 2] = p[64 * G4 + 32 + cc];
}

template <int NT, bool SYM, int PG, bool F32>
__device__ __forceinline__ void gram_wave(const float* X1, int ld1, const float* X2, int ld2, int vec, int64_t r0,
                                          int64_t r1, int64_t rows, int half, int l, double* out, double* lds) {
  constexpr int NP = npairs(NT, SYM);
  constexpr int PPW = (NP - PG + 3) / 4;  // pairs p = PG + 4q
  const int lane = threadIdx.x & 63;
  const int kr = lane >> 4, cc = lane & 15;
  d4 acc[PPW > 0 ? PPW : 1];
  f4 acc32[PPW > 0 ? PPW : 1];
#pragma unroll
  for (int q = 0; q < (PPW > 0 ? PPW : 1); ++q) {
    acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    acc32[q] = f4{0.f, 0.f, 0.f, 0.f};
  }
  int steps = 0;
  // one step: the 4 rows in xa (and xb) enter every tile pair of this wave
  auto step = [&](const float* xa, const float* xb) {
    double a[NT], b[NT];
    float a32[NT], b32[NT];
#pragma unroll
    for (int I = 0; I < NT; ++I) {
      if constexpr (F32) {
        a32[I] = xa[I];
        if constexpr (!SYM) b32[I] = xb[I];
      } else {
        a[I] = (double)xa[I];
        if constexpr (!SYM) b[I] = (double)xb[I];
      }
    }
    static_for<0, PPW>([&](auto qc) {
      constexpr int p = PG + 4 * decltype(qc)::value;
      constexpr int I = pair_i(NT, SYM, p), J = pair_j(NT, SYM, p);
      if constexpr (F32) {
        if constexpr (SYM) acc32[qc] = __builtin_amdgcn_mfma_f32_16x16x4f32(a32[I], a32[J], acc32[qc], 0, 0, 0);
        else acc32[qc] = __builtin_amdgcn_mfma_f32_16x16x4f32(a32[I], b32[J], acc32[qc], 0, 0, 0);
      } else {
        if constexpr (SYM) acc[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], a[J], acc[qc], 0, 0, 0);
        else acc[qc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], b[J], acc[qc], 0, 0, 0);
      }
    });
    if constexpr (F32) {
      if (++steps == kFlushSteps) {
        steps = 0;
        static_for<0, PPW>([&](auto qc) {
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[qc][e] += (double)acc32[qc][e];
          acc32[qc] = f4{0.f, 0.f, 0.f, 0.f};
        });
      }
    }
  };
  int64_t r = r0 + 4 * half;
  if (kGramRing > 0 && (vec == 2 || (vec == 3 && r1 < rows)) && r1 > r0 && ((r1 - r0) & 7) == 0) {
    // every step of the stretch is full: a ring of kGramRing row buffers, each refilled
    // kGramRing - 1 steps before its step, with a wave-uniform step count
    constexpr int D = kGramRing > 0 ? kGramRing : 1;
    float ra[D][NT], rb[D][NT];
    const int64_t nsteps = (r1 - r0) / 8;
    static_for<0, D - 1>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      gram_load_wide<NT>(X1, ld1, r + 8 * u + kr, r1, cc, ra[u]);
      if constexpr (!SYM) gram_load_wide<NT>(X2, ld2, r + 8 * u + kr, r1, cc, rb[u]);
    });
    for (int64_t i = 0; i < nsteps; i += D) {
      static_for<0, D>([&](auto uc) {
        constexpr int u = decltype(uc)::value;
        constexpr int un = (u + D - 1) % D;
        const int64_t rn = r + 8 * (i + u + D - 1) + kr;
        gram_load_wide<NT>(X1, ld1, rn, r1, cc, ra[un]);
        if constexpr (!SYM) gram_load_wide<NT>(X2, ld2, rn, r1, cc, rb[un]);
        if (i + u < nsteps) step(ra[u], rb[u]);
      });
    }
  } else {
    float na[NT], nb[NT], ca[NT], cb[NT];
    if (r < r1) {
      gram_load<NT>(X1, ld1, r + kr, r + kr < r1, l, cc, vec != 0, na);
      if constexpr (!SYM) gram_load<NT>(X2, ld2, r + kr, r + kr < r1, l, cc, vec != 0, nb);
    }
    for (; r < r1; r += 8) {
#pragma unroll
      for (int I = 0; I < NT; ++I) {
        ca[I] = na[I];
        if constexpr (!SYM) cb[I] = nb[I];
      }
      // the next step's rows load while this step's MFMAs run
      const int64_t rn = r + 8;
      if (rn < r1) {
        gram_load<NT>(X1, ld1, rn + kr, rn + kr < r1, l, cc, vec != 0, na);
        if constexpr (!SYM) gram_load<NT>(X2, ld2, rn + kr, rn + kr < r1, l, cc, vec != 0, nb);
      }
      step(ca, cb);
    }
  }
  if constexpr (F32) {
    static_for<0, PPW>([&](auto qc) {
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[qc][e] += (double)acc32[qc][e];
    });
  }
  // the two row streams combine in LDS (second stream first, fixed order)
  if (half == 1) {
    static_for<0, PPW>([&](auto qc) {
      double* o = lds + ((size_t)(PG + 4 * decltype(qc)::value) * 64 + lane) * 4;
      o[0] = acc[qc][0];
      o[1] = acc[qc][1];
      o[2] = acc[qc][2];
      o[3] = acc[qc][3];
    });
  }
  __syncthreads();
  if (half == 0) {
    static_for<0, PPW>([&](auto qc) {
      constexpr int p = PG + 4 * decltype(qc)::value;
      const double* i2 = lds + ((size_t)p * 64 + lane) * 4;
      double* o = out + (size_t)p * 256 + lane * 4;
      o[0] = acc[qc][0] + i2[0];
      o[1] = acc[qc][1] + i2[1];
      o[2] = acc[qc][2] + i2[2];
      o[3] = acc[qc][3] + i2[3];
    });
  }
}

template <int NT, bool SYM, bool F32>
__global__ __launch_bounds__(kGramThreads) void gram_kernel(const float* X1, int ld1, const float* X2, int ld2,
                                                            int vec, int64_t rows, int l, int64_t rows_per_block,
                                                            double* partial) {
  constexpr int NP = npairs(NT, SYM);
  __shared__ double lds[NP * 256];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(rows, r0 + rows_per_block);
  double* out = partial + (size_t)blockIdx.x * NP * 256;
  // the wave index as a scalar: the row loops and the tile-group switch branch uniformly
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), half = w >> 2;
  switch (w & 3) {
    case 0: gram_wave<NT, SYM, 0, F32>(X1, ld1, X2, ld2, vec, r0, r1, rows, half, l, out, lds); break;
    case 1: gram_wave<NT, SYM, 1, F32>(X1, ld1, X2, ld2, vec, r0, r1, rows, half, l, out, lds); break;
    case 2: gram_wave<NT, SYM, 2, F32>(X1, ld1, X2, ld2, vec, r0, r1, rows, half, l, out, lds); break;
    default: gram_wave<NT, SYM, 3, F32>(X1, ld1, X2, ld2, vec, r0, r1, rows, half, l, out, lds); break;
  }
}

// Sum of the block partials: kRedEnt consecutive entries per workgroup, kRedPart interleaved
// block streams per entry (stream s adds blocks s, s + kRedPart, ... in order), combined in a
// fixed order; then the entry goes to its place in G (tile columns mapped back, both
// triangles for SYM).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* partial, int nblk, int nt, bool sym,
                                                          bool f32_layout, int l, double* G, int ldg) {
  __shared__ double red[kRedPart][kRedEnt];
  const int np = sym ? nt * (nt + 1) / 2 : nt * nt;
  const int x = threadIdx.x % kRedEnt, part = threadIdx.x / kRedEnt;
  const int e = blockIdx.x * kRedEnt + x;
  double s = 0.0;
  if (e < np * 256) {
#pragma unroll 8
    for (int b = part; b < nblk; b += kRedPart) s += partial[(size_t)b * np * 256 + e];
  }
  red[part][x] = s;
  __syncthreads();
  if (part != 0 || e >= np * 256) return;
  s = 0.0;
#pragma unroll
  for (int q = 0; q < kRedPart; ++q) s += red[q][x];
  const int p = e >> 8, t = e & 255, lane = t >> 2, r = t & 3;
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
  const int i = gram_col(nt, I, f32_layout ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r);
  const int j = gram_col(nt, J, lane & 15);
  if (i >= l || j >= l) return;
  if (sym) {
    if (I == J && i > j) return;
    G[(size_t)i * ldg + j] = s;
    G[(size_t)j * ldg + i] = s;
  } else {
    G[(size_t)i * ldg + j] = s;
  }
}

template <bool SYM, bool F32>
void gram_dispatch(int nt, unsigned grid, const float* X1, int ld1, const float* X2, int ld2, int vec, int64_t rows,
                   int l, int64_t rpb, double* partial, hipStream_t st) {
  switch (nt) {
    case 2: gram_kernel<2, SYM, F32><<<grid, kGramThreads, 0, st>>>(X1, ld1, X2, ld2, vec, rows, l, rpb, partial); break;
    case 3: gram_kernel<3, SYM, F32><<<grid, kGramThreads, 0, st>>>(X1, ld1, X2, ld2, vec, rows, l, rpb, partial); break;
    case 4: gram_kernel<4, SYM, F32><<<grid, kGramThreads, 0, st>>>(X1, ld1, X2, ld2, vec, rows, l, rpb, partial); break;
    case 6: gram_kernel<6, SYM, F32><<<grid, kGramThreads, 0, st>>>(X1, ld1, X2, ld2, vec, rows, l, rpb, partial); break;
    case 7: gram_kernel<7, SYM, F32><<<grid, kGramThreads, 0, st>>>(X1, ld1, X2, ld2, vec, rows, l, rpb, partial); break;
    default: gram_kernel<8, SYM, F32><<<grid, kGramThreads, 0, st>>>(X1, ld1, X2, ld2, vec, rows, l, rpb, partial); break;
  }
}

}  // namespace

size_t gram_partial_bytes(int /*l*/) { return (size_t)kGramMaxBlocks * kMaxPairs * 256 * sizeof(double); }

void launch_gram(const void* X1, bool /*bf16*/, int ld1, const float* X2, int ld2, int64_t rows, int l,
                 double* partial, double* G, int ldg, hipStream_t st, bool f32_mfma) {
  // tiles of 16 columns: 1 and 5 round up to a trailing pair (2, 6); 3 and 7 end with a pair
  // and a single tile
  int nt = (l + 15) / 16;
  if (nt % 4 == 1) ++nt;
  const int ext = 16 * nt;
  const bool sym = (X2 == nullptr);
  const float* x1 = static_cast<const float*>(X1);
  auto aligned = [](const float* x, int ld) { return (ld % 4) == 0 && (reinterpret_cast<uintptr_t>(x) % 16) == 0; };
  // 2: aligned rows whose leading dimension covers every tile column; 3: aligned rows whose
  // tile columns end inside the next row (unconditional loads in every block but the last);
  // 1: aligned rows; 0: element loads
  int vec = aligned(x1, ld1) && (sym || aligned(X2, ld2)) ? 1 : 0;
  if (vec && ld1 >= ext && (sym || ld2 >= ext)) vec = 2;
  else if (vec && 2 * ld1 >= ext && (sym || 2 * ld2 >= ext)) vec = 3;
  int64_t grid = (rows + 127) / 128;
  if (grid > kGramMaxBlocks) grid = kGramMaxBlocks;
  if (grid < 1) grid = 1;
  int64_t rpb = (rows + grid - 1) / grid;
  rpb = (rpb + 7) / 8 * 8;
  const bool f32 = f32_mfma && sym;  // the FP32 variant serves the symmetric Gram of eigSVD only
  if (f32) gram_dispatch<true, true>(nt, (unsigned)grid, x1, ld1, x1, ld1, vec, rows, l, rpb, partial, st);
  else if (sym) gram_dispatch<true, false>(nt, (unsigned)grid, x1, ld1, x1, ld1, vec, rows, l, rpb, partial, st);
  else gram_dispatch<false, false>(nt, (unsigned)grid, x1, ld1, X2, ld2, vec, rows, l, rpb, partial, st);
  const int np = sym ? nt * (nt + 1) / 2 : nt * nt;
  gram_reduce_kernel<<<(unsigned)((np * 256 + kRedEnt - 1) / kRedEnt), 256, 0, st>>>(partial, (int)grid, nt, sym, f32,
                                                                                   l, G, ldg);
}

}  // namespace frpca
