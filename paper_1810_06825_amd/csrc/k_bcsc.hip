// Blocked column-major order for the transpose product A^T Y when the gathered panel Y is
// too large for the caches (Alg. 6: Y is m x l with m >> n).
//
// In plain column order, each nonzero of A^T Y gathers a whole row of Y and the ~nnz/m
// nonzeros that share a row of Y are far apart in time, so every gather misses the caches.
// Frequent ("hot") columns are therefore split by row block: their nonzeros are ordered by
// (row block, hot column, row), so all hot columns sweep one block of Y rows (4096 rows,
// 2 MB at l = 128) while it sits in L2, each (row block, hot column) pair being one merge-path
// segment whose sum is a partial row. The remaining ("tail") columns keep one segment each.
// A combine kernel adds the partials of each hot column over the row blocks in a fixed order,
// so the product stays deterministic.
//
// A column is hot when it holds at least kHotPerBlock nonzeros per row block on average, so
// every partial row amortizes its write over that many gathers. Segment order: the nblk x H
// hot segments (row block major), then one segment per tail column. The two parts run as
// separate merge-path launches: the hot one sweeps the row blocks in order, each XCD taking
// its own chunks of partitions one after another from a counter, so its gathers hit L2, and the tail's random-row gathers, which would
// evict those blocks, come afterwards and write their rows of the result directly (the plan
// maps tail segment i to column tailcol[i]).
#include "kernels.h"

namespace frpca {
namespace {

__global__ void hot_flags_kernel(const int32_t* cp, int64_t n, int32_t thresh, int32_t* hot, int32_t* tail) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t h = (cp[i + 1] - cp[i]) >= thresh ? 1 : 0;
  hot[i] = h;
  tail[i] = 1 - h;
}

__global__ void colmap_kernel(const int32_t* hot, const int32_t* hpre, const int32_t* tpre, int64_t n,
                              int32_t* colmap) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  colmap[i] = hot[i] ? hpre[i] : -1 - tpre[i];
}

// Segment pointers of the tail part, rebased to its first nonzero.
__global__ void rebase_kernel(const int32_t* ptr, int64_t count, int32_t base, int32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) out[i] = ptr[i] - base;
}

// Inverse maps of colmap: hot index -> column, tail index -> column.
__global__ void colmap_inverse_kernel(const int32_t* colmap, int64_t n, int32_t* hotcol, int32_t* tailcol) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  const int32_t cm = colmap[c];
  if (cm >= 0) hotcol[cm] = (int32_t)c;
  else tailcol[-1 - cm] = (int32_t)c;
}

// One block per hot column: wave q sums the partial rows of row blocks q, q + 8, q + 16, ...
// and wave 0 adds the eight sums in wave order, so the result does not depend on timing. A
// lane owns columns 2 lane and 2 lane + 1.
constexpr int kCombWaves = 8;
__global__ __launch_bounds__(64 * kCombWaves) void combine_hot_kernel(const float* P, int ldp, const int32_t* hotcol,
                                                                     int64_t hot_cols, int64_t nblk, int lp,
                                                                     float* X32, uint16_t* X16, int ldx,
                                                                     const float* csub_v, const float* csub_s) {
  __shared__ float2 red[kCombWaves][64];
  const int64_t hc = blockIdx.x;
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = 2 * lane;
  float2 s = make_float2(0.f, 0.f);
  if (col < lp) {
#pragma unroll 4
    for (int64_t b = q; b < nblk; b += kCombWaves) {
      const float2 v = *reinterpret_cast<const float2*>(P + (size_t)(b * hot_cols + hc) * ldp + col);
      s.x += v.x;
      s.y += v.y;
    }
  }
  red[q][lane] = s;
  __syncthreads();
  if (q == 0 && col < lp) {
    float2 tot = red[0][lane];
#pragma unroll
    for (int r = 1; r < kCombWaves; ++r) {
      tot.x += red[r][lane].x;
      tot.y += red[r][lane].y;
    }
    const int64_t orow = hotcol[hc];
    if (csub_v) {
      const float sc = csub_s ? csub_s[orow] : 1.f;
      tot.x -= sc * csub_v[col];
      tot.y -= sc * csub_v[col + 1];
    }
    const size_t o = (size_t)orow * ldx + col;
    if (X32) store2_f32(X32, o, tot);
    if (X16) store2_bf16(X16, o, tot);
  }
}

}  // namespace

void launch_hot_flags(const int32_t* cp, int64_t n, int32_t thresh, int32_t* hot, int32_t* tail, hipStream_t st) {
  if (n <= 0) return;
  hot_flags_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(cp, n, thresh, hot, tail);
}

void launch_colmap(const int32_t* hot, const int32_t* hpre, const int32_t* tpre, int64_t n, int32_t* colmap,
                   hipStream_t st) {
  if (n <= 0) return;
  colmap_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(hot, hpre, tpre, n, colmap);
}

void launch_rebase(const int32_t* ptr, int64_t count, int32_t base, int32_t* out, hipStream_t st) {
  if (count <= 0) return;
  rebase_kernel<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(ptr, count, base, out);
}

void launch_colmap_inverse(const int32_t* colmap, int64_t n, int32_t* hotcol, int32_t* tailcol, hipStream_t st) {
  if (n <= 0) return;
  colmap_inverse_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(colmap, n, hotcol, tailcol);
}

void launch_bcsc_combine(const float* P, int ldp, const int32_t* hotcol, int64_t hot_cols, int64_t nblk, int lp,
                         float* X32, uint16_t* X16, int ldx, hipStream_t st, SpmmCorr corr) {
  if (hot_cols <= 0) return;
  combine_hot_kernel<<<(unsigned)hot_cols, 64 * kCombWaves, 0, st>>>(P, ldp, hotcol, hot_cols, nblk, lp, X32, X16,
                                                                      ldx, corr.v, corr.s);
}

}  // namespace frpca
