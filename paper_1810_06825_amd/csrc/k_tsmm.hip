// Tall-skinny panel times small matrix, out = X B, on the FP64 matrix cores.
//
// Used for every "X times an l x l (or l x k) matrix" step of the method: the eigSVD basis
// U = X V diag(1/S) (Alg. 2 step 5), the LU basis P^T L = X U^-1 (eq. 8), the final
// U = Z W(:,ind) diag(1/S(ind)) and V = Q W(:,ind) of Alg. 5/6, and the adjoint's panels.
// B (<= 128 x 128, FP64) sits in LDS; a wave computes a 16-row strip of out as NCT 16x16
// tiles with v_mfma_f64_16x16x4f64: lane l supplies X[r0 + l%16][4t + l/16] as the A operand
// and B[4t + l/16][16j + l%16] as the B operand of k-step t; value q of its result is row
// l/16 + 4q, column l%16 (layout checked on gfx950). FP32 (or BF16) inputs are widened exactly to FP64.
// An FP32 form (B rounded to FP32, v_mfma_f32_16x16x4f32 at twice the FP64 rate, value q of a
// lane's result in row 4 (l/16) + q) serves products whose coefficient matrix is well
// conditioned, where FP32 accumulation costs about one FP32 rounding per term.
#include <type_traits>

#include "kernels.h"

namespace frpca {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 8 waves per block share one copy of B in LDS (up to 133 KB, so one block per CU): two waves
// per SIMD hide the panel-load latency behind the other's MFMAs.
constexpr int kTsmmThreads = 512;
constexpr int kTsmmWaves = kTsmmThreads / 64;

struct TsmmArgs {
  const void* X;
  int ldx;
  int64_t rows;
  int kdim;
  const double* B;
  int ldb;
  int c;      // valid output columns
  int c_out;  // output columns written (c..c_out-1 are zero)
  float* out;
  int ldo;
  uint16_t* out_bf16;
  int ldo16;
  int vec;    // rows of X allow 4-wide vector loads
  const float* y2;   // optional second term y2 diag(d2): out += y2[r, c] d2[c, c]
  int ldy2;
  const double* d2;
  int ldd2;
};

// k is visited in groups of 16: lane l (group j = l/16, row lr = l%16) loads the four
// consecutive entries X[r0 + lr][16u + 4j .. 16u + 4j + 3] with one vector load and feeds them
// to four k-steps (v = 0..3); k-step (u, v) covers k = 16u + 4j + v over j, and the B operand
// lane supplies B[16u + 4j + v][16 jc + lr] from LDS. The next tile's row slab is fetched
// into registers while the current tile's MFMAs run.
template <bool BF16>
__device__ __forceinline__ void load4(const TsmmArgs& a, int64_t row, int k0, float v[4]) {
  const bool rok = row < a.rows;
  if (a.vec && rok && k0 + 3 < a.kdim) {
    if constexpr (BF16) {
      const uint2 w = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(a.X) + (size_t)row * a.ldx + k0);
      v[0] = bf16_to_f32((uint16_t)(w.x & 0xFFFF));
      v[1] = bf16_to_f32((uint16_t)(w.x >> 16));
      v[2] = bf16_to_f32((uint16_t)(w.y & 0xFFFF));
      v[3] = bf16_to_f32((uint16_t)(w.y >> 16));
    } else {
      const float4 w = *reinterpret_cast<const float4*>(static_cast<const float*>(a.X) + (size_t)row * a.ldx + k0);
      v[0] = w.x;
      v[1] = w.y;
      v[2] = w.z;
      v[3] = w.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float x = 0.f;
      if (rok && k0 + q < a.kdim) {
        if constexpr (BF16) x = bf16_to_f32(static_cast<const uint16_t*>(a.X)[(size_t)row * a.ldx + k0 + q]);
        else x = static_cast<const float*>(a.X)[(size_t)row * a.ldx + k0 + q];
      }
      v[q] = x;
    }
  }
}

// Branch-free form for vector-aligned panels: the row is clamped into the panel and a group past
// the row's end reads the row's first columns (k0 and ldx are multiples of 4, so the load stays
// in the row); the caller zeroes entries past kdim. With no load under a lane-dependent branch,
// the compiler keeps each refill where it is written and waits only for the loads it uses.
template <bool BF16>
__device__ __forceinline__ void load4_nb(const TsmmArgs& a, int64_t row, int k0, float v[4]) {
  const size_t o = (size_t)(row < a.rows ? row : a.rows - 1) * a.ldx + (k0 < a.ldx ? k0 : 0);
  if constexpr (BF16) {
    const uint2 w = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(a.X) + o);
    v[0] = bf16_to_f32((uint16_t)(w.x & 0xFFFF));
    v[1] = bf16_to_f32((uint16_t)(w.x >> 16));
    v[2] = bf16_to_f32((uint16_t)(w.y & 0xFFFF));
    v[3] = bf16_to_f32((uint16_t)(w.y >> 16));
  } else {
    const float4 w = *reinterpret_cast<const float4*>(static_cast<const float*>(a.X) + o);
    v[0] = w.x;
    v[1] = w.y;
    v[2] = w.z;
    v[3] = w.w;
  }
}

template <int NKT, int NCT, bool BF16, bool VEC, bool F32>
__global__ __launch_bounds__(kTsmmThreads) void tsmm_kernel(TsmmArgs a) {
  using T = typename std::conditional<F32, float, double>::type;
  using TV = typename std::conditional<F32, f4, d4>::type;
  constexpr int KP = NKT * 4;
  constexpr int NU = KP / 16;     // groups of 16 k
  constexpr int CP = NCT * 16;
  // pad rows so the 4 k-rows of an operand fetch use distinct banks
  constexpr int LDS_LD = F32 ? CP + 4 : CP + 2;
  __shared__ T Bs[KP * LDS_LD];
  __shared__ T Ds[CP];  // diagonal of d2 (second term)
  for (int i = threadIdx.x; i < KP * CP; i += kTsmmThreads) {
    const int r = i / CP, cc = i - r * CP;
    Bs[r * LDS_LD + cc] = (r < a.kdim && cc < a.c) ? (T)a.B[(size_t)r * a.ldb + cc] : (T)0;
  }
  if (a.y2)
    for (int i = threadIdx.x; i < CP; i += kTsmmThreads) Ds[i] = i < a.c ? (T)a.d2[(size_t)i * a.ldd2 + i] : (T)0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t ntiles = (a.rows + 15) / 16;
  const int64_t wstride = (int64_t)gridDim.x * kTsmmWaves;
  int64_t tile = (int64_t)blockIdx.x * kTsmmWaves + (threadIdx.x >> 6);
  float xs[NU][4];
  if (VEC || tile < ntiles) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if constexpr (VEC) load4_nb<BF16>(a, tile * 16 + lr, 16 * u + 4 * lk, xs[u]);
      else load4<BF16>(a, tile * 16 + lr, 16 * u + 4 * lk, xs[u]);
    }
  }
  for (; tile < ntiles; tile += wstride) {
    const int64_t r0 = tile * 16;
    const int64_t nxt = tile + wstride;
    TV acc[NCT];
#pragma unroll
    for (int j = 0; j < NCT; ++j) acc[j] = TV{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      T av[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if constexpr (VEC) av[v] = (16 * u + 4 * lk + v < a.kdim) ? (T)xs[u][v] : (T)0;
        else av[v] = (T)xs[u][v];
      }
      // this group's registers now refill with the next tile's slab (past the last tile the
      // branch-free form reads the panel's last row, unused)
      if constexpr (VEC) load4_nb<BF16>(a, nxt * 16 + lr, 16 * u + 4 * lk, xs[u]);
      else if (nxt < ntiles) load4<BF16>(a, nxt * 16 + lr, 16 * u + 4 * lk, xs[u]);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T* brow = Bs + (16 * u + 4 * lk + v) * LDS_LD + lr;
#pragma unroll
        for (int j = 0; j < NCT; ++j) {
          if constexpr (F32) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[v], brow[16 * j], acc[j], 0, 0, 0);
          else acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[v], brow[16 * j], acc[j], 0, 0, 0);
        }
      }
      // keep each group's LDS operand reads next to their MFMAs (hoisting them all would
      // exhaust the register file)
      __builtin_amdgcn_sched_barrier(0);
    }
    if (a.y2) {
      // the second term's entries, all loaded before any is used (row and column clamped
      // into the panel; the clamped ones meet a zero in Ds or are not stored)
      float yv[NCT][4];
#pragma unroll
      for (int j = 0; j < NCT; ++j) {
        const int col = 16 * j + lr;
        const int cl = col < a.c ? col : a.c - 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t row = r0 + (F32 ? 4 * lk + q : lk + 4 * q);
          const int64_t rl = row < a.rows ? row : a.rows - 1;
          yv[j][q] = a.y2[(size_t)rl * a.ldy2 + cl];
        }
      }
#pragma unroll
      for (int j = 0; j < NCT; ++j) {
        const T dj = Ds[16 * j + lr];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[j][q] += (T)yv[j][q] * dj;
      }
    }
#pragma unroll
    for (int j = 0; j < NCT; ++j) {
      const int col = 16 * j + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = r0 + (F32 ? 4 * lk + q : lk + 4 * q);
        if (row < a.rows && col < a.c_out) {
          const T t = acc[j][q];
          float v = (col < a.c) ? (float)t : 0.0f;
          if (a.out) a.out[(size_t)row * a.ldo + col] = v;
          if (a.out_bf16) a.out_bf16[(size_t)row * a.ldo16 + col] = f32_to_bf16(v);
        }
      }
    }
  }
}

template <int NKT, bool BF16, bool VEC, bool F32>
void tsmm_dispatch_c(int nct, unsigned grid, const TsmmArgs& a, hipStream_t st) {
  switch (nct) {
    case 1: tsmm_kernel<NKT, 1, BF16, VEC, F32><<<grid, kTsmmThreads, 0, st>>>(a); break;
    case 2: tsmm_kernel<NKT, 2, BF16, VEC, F32><<<grid, kTsmmThreads, 0, st>>>(a); break;
    case 3: tsmm_kernel<NKT, 3, BF16, VEC, F32><<<grid, kTsmmThreads, 0, st>>>(a); break;
    case 4: tsmm_kernel<NKT, 4, BF16, VEC, F32><<<grid, kTsmmThreads, 0, st>>>(a); break;
    case 5: tsmm_kernel<NKT, 5, BF16, VEC, F32><<<grid, kTsmmThreads, 0, st>>>(a); break;
    case 6: tsmm_kernel<NKT, 6, BF16, VEC, F32><<<grid, kTsmmThreads, 0, st>>>(a); break;
    case 7: tsmm_kernel<NKT, 7, BF16, VEC, F32><<<grid, kTsmmThreads, 0, st>>>(a); break;
    default: tsmm_kernel<NKT, 8, BF16, VEC, F32><<<grid, kTsmmThreads, 0, st>>>(a); break;
  }
}

template <bool BF16, bool VEC, bool F32 = false>
void tsmm_dispatch(int nkt, int nct, unsigned grid, const TsmmArgs& a, hipStream_t st) {
  // k extents are rounded up to 32, 64, 96, 112 or 128 (k-steps of 4 in groups of 16);
  // vector loads need 16-byte (FP32) or 8-byte (BF16) aligned rows, which the dispatcher checks
  if (nkt <= 8) tsmm_dispatch_c<8, BF16, VEC, F32>(nct, grid, a, st);
  else if (nkt <= 16) tsmm_dispatch_c<16, BF16, VEC, F32>(nct, grid, a, st);
  else if (nkt <= 24) tsmm_dispatch_c<24, BF16, VEC, F32>(nct, grid, a, st);
  else if (nkt <= 28) tsmm_dispatch_c<28, BF16, VEC, F32>(nct, grid, a, st);
  else tsmm_dispatch_c<32, BF16, VEC, F32>(nct, grid, a, st);
}

}  // namespace

void launch_tsmm(const void* X, bool x_bf16, int ldx, int64_t rows, int kdim, const double* B, int ldb, int c,
                 int c_out, float* out, int ldo, uint16_t* out_bf16, int ldo16, hipStream_t st,
                 const float* y2, int ldy2, const double* d2, int ldd2, bool f32_mfma) {
  if (rows <= 0 || c_out <= 0) return;
  const uintptr_t xa = reinterpret_cast<uintptr_t>(X);
  const int vec = x_bf16 ? ((ldx % 4) == 0 && (xa % 8) == 0) : ((ldx % 4) == 0 && (xa % 16) == 0);
  TsmmArgs a{X, ldx, rows, kdim, B, ldb, c, c_out, out, ldo, out_bf16, ldo16, vec,
             y2, ldy2, d2, ldd2};
  const int nkt = (kdim + 3) / 4;
  const int nct = (c_out + 15) / 16;
  const int64_t ntiles = (rows + 15) / 16;
  // one persistent block per compute unit (B in LDS allows only one): B is staged once per CU
  // and every wave walks several tiles, so the next-tile prefetch keeps the MFMAs fed
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  int64_t grid = (ntiles + kTsmmWaves - 1) / kTsmmWaves;
  if (grid > cus) grid = cus;
  if (f32_mfma && !x_bf16) {
    if (vec) tsmm_dispatch<false, true, true>(nkt, nct, (unsigned)grid, a, st);
    else tsmm_dispatch<false, false, true>(nkt, nct, (unsigned)grid, a, st);
  } else if (x_bf16) {
    if (vec) tsmm_dispatch<true, true>(nkt, nct, (unsigned)grid, a, st);
    else tsmm_dispatch<true, false>(nkt, nct, (unsigned)grid, a, st);
  } else {
    if (vec) tsmm_dispatch<false, true>(nkt, nct, (unsigned)grid, a, st);
    else tsmm_dispatch<false, false>(nkt, nct, (unsigned)grid, a, st);
  }
}

}  // namespace frpca
