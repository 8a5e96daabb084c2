// Tall-skinny panel times small matrix, out = X B, on the FP64 matrix cores.
//
// Used for every "X times an l x l (or l x k) matrix" step of the method: the eigSVD basis
// U = X V diag(1/S) (Alg. 2 step 5), the LU basis P^T L = X U^-1 (eq. 8), the final
// U = Z W(:,ind) diag(1/S(ind)) and V = Q W(:,ind) of Alg. 5/6, and the adjoint's panels.
// B (<= 128 x 128, FP64) sits in LDS; a wave computes a 16-row strip of out as NCT 16x16
// tiles with v_mfma_f64_16x16x4f64: lane l supplies X[r0 + l%16][4t + l/16] as the A operand
// and B[4t + l/16][16j + l%16] as the B operand of k-step t; value q of its result is row
// l/16 + 4q, column l%16 (layout checked on gfx950). FP32 (or BF16) inputs are widened exactly to FP64.
#include "kernels.h"

namespace frpca {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

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
  int accumulate;
};

template <int NKT, int NCT, bool BF16>
__global__ __launch_bounds__(256) void tsmm_kernel(TsmmArgs a) {
  constexpr int KP = NKT * 4;
  constexpr int CP = NCT * 16;
  constexpr int LDS_LD = CP + 2;  // pad rows so the 4 k-rows of an operand fetch use distinct banks
  __shared__ double Bs[KP * LDS_LD];
  for (int i = threadIdx.x; i < KP * CP; i += 256) {
    const int r = i / CP, cc = i - r * CP;
    Bs[r * LDS_LD + cc] = (r < a.kdim && cc < a.c) ? a.B[(size_t)r * a.ldb + cc] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t ntiles = (a.rows + 15) / 16;
  const int64_t wstride = (int64_t)gridDim.x * 4;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles; tile += wstride) {
    const int64_t r0 = tile * 16;
    const int64_t ra = r0 + lr;
    const bool rok = ra < a.rows;
    d4 acc[NCT];
#pragma unroll
    for (int j = 0; j < NCT; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int t = 0; t < NKT; ++t) {
      const int k = 4 * t + lk;
      double av = 0.0;
      if (rok && k < a.kdim) {
        if constexpr (BF16) av = (double)bf16_to_f32(static_cast<const uint16_t*>(a.X)[(size_t)ra * a.ldx + k]);
        else av = (double)static_cast<const float*>(a.X)[(size_t)ra * a.ldx + k];
      }
      const double* brow = Bs + k * LDS_LD + lr;
#pragma unroll
      for (int j = 0; j < NCT; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, brow[16 * j], acc[j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NCT; ++j) {
      const int col = 16 * j + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = r0 + lk + 4 * q;
        if (row < a.rows && col < a.c_out) {
          float v = (col < a.c) ? (float)acc[j][q] : 0.0f;
          if (a.out) {
            float* o = a.out + (size_t)row * a.ldo + col;
            if (a.accumulate && col < a.c) v = (float)((double)*o + acc[j][q]);
            *o = v;
          }
          if (a.out_bf16) a.out_bf16[(size_t)row * a.ldo16 + col] = f32_to_bf16(v);
        }
      }
    }
  }
}

template <int NKT, bool BF16>
void tsmm_dispatch_c(int nct, unsigned grid, const TsmmArgs& a, hipStream_t st) {
  switch (nct) {
    case 1: tsmm_kernel<NKT, 1, BF16><<<grid, 256, 0, st>>>(a); break;
    case 2: tsmm_kernel<NKT, 2, BF16><<<grid, 256, 0, st>>>(a); break;
    case 3: tsmm_kernel<NKT, 3, BF16><<<grid, 256, 0, st>>>(a); break;
    case 4: tsmm_kernel<NKT, 4, BF16><<<grid, 256, 0, st>>>(a); break;
    case 5: tsmm_kernel<NKT, 5, BF16><<<grid, 256, 0, st>>>(a); break;
    case 6: tsmm_kernel<NKT, 6, BF16><<<grid, 256, 0, st>>>(a); break;
    case 7: tsmm_kernel<NKT, 7, BF16><<<grid, 256, 0, st>>>(a); break;
    default: tsmm_kernel<NKT, 8, BF16><<<grid, 256, 0, st>>>(a); break;
  }
}

template <bool BF16>
void tsmm_dispatch(int nkt, int nct, unsigned grid, const TsmmArgs& a, hipStream_t st) {
  // k extents are rounded up to multiples of 32 (8 k-steps of 4)
  if (nkt <= 8) tsmm_dispatch_c<8, BF16>(nct, grid, a, st);
  else if (nkt <= 16) tsmm_dispatch_c<16, BF16>(nct, grid, a, st);
  else if (nkt <= 24) tsmm_dispatch_c<24, BF16>(nct, grid, a, st);
  else tsmm_dispatch_c<32, BF16>(nct, grid, a, st);
}

}  // namespace

void launch_tsmm(const void* X, bool x_bf16, int ldx, int64_t rows, int kdim, const double* B, int ldb, int c,
                 int c_out, float* out, int ldo, uint16_t* out_bf16, int ldo16, bool accumulate, hipStream_t st) {
  if (rows <= 0 || c_out <= 0) return;
  TsmmArgs a{X, ldx, rows, kdim, B, ldb, c, c_out, out, ldo, out_bf16, ldo16, accumulate ? 1 : 0};
  const int nkt = (kdim + 3) / 4;
  const int nct = (c_out + 15) / 16;
  const int64_t ntiles = (rows + 15) / 16;
  int64_t grid = (ntiles + 3) / 4;
  if (grid > 2048) grid = 2048;
  if (x_bf16) tsmm_dispatch<true>(nkt, nct, (unsigned)grid, a, st);
  else tsmm_dispatch<false>(nkt, nct, (unsigned)grid, a, st);
}

}  // namespace frpca
