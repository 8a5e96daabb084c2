// Setup of the column-major mirror (frpca_create): CSR validation, 32-bit pointers, row
// expansion, stable LSD radix sort of the nonzeros by column, exclusive scans, gathers and
// the merge-path partition tables of both products. Integer work, deterministic.
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;  // 2048 values per scan block

constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixRounds = 32;
constexpr int kRadixTile = kWave * kRadixRounds;    // 2048 keys per single-wave tile

// ---------------------------------------------------------------- validation
__global__ __launch_bounds__(256) void validate_rows_kernel(int64_t m, int64_t n, int64_t nnz,
                                                            const int64_t* rp, const int32_t* col,
                                                            int* flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > m) return;
  if (r == 0 && rp[0] != 0) atomicOr(flag, 1);
  if (r == m) {
    if (rp[m] != nnz) atomicOr(flag, 1);
    return;
  }
  const int64_t a = rp[r], b = rp[r + 1];
  if (b < a) {
    atomicOr(flag, 2);
    return;
  }
  if (a < 0 || b > nnz) {
    atomicOr(flag, 1);
    return;
  }
  int prev = -1;
  for (int64_t e = a; e < b; ++e) {
    const int c = col[e];
    if (c < 0 || c >= n) {
      atomicOr(flag, 4);
      return;
    }
    if (c <= prev) {
      atomicOr(flag, 8);
      return;
    }
    prev = c;
  }
}

__global__ __launch_bounds__(256) void validate_vals_kernel(int64_t nnz, const float* val, int* flag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz && !isfinite(val[e])) atomicOr(flag, 16);
}

__global__ __launch_bounds__(256) void ptr_to_i32_kernel(const int64_t* p, int64_t count, int32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (int32_t)p[i];
}

// row_of[e] = r with rp[r] <= e < rp[r+1] (binary search; rows may be empty).
__global__ __launch_bounds__(256) void expand_rows_kernel(const int32_t* rp, int64_t m, int64_t nnz,
                                                          int32_t* row_of) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int64_t lo = 0, hi = m - 1;  // largest r with rp[r] <= e
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (rp[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  row_of[e] = (int32_t)lo;
}

// ---------------------------------------------------------------- exclusive scan
__global__ __launch_bounds__(kScanBlock) void scan_tiles_kernel(const int32_t* in, int32_t* out,
                                                                int64_t count, int32_t* tile_sums) {
  __shared__ int32_t part[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < count) ? in[base + i] : 0;
    s += v[i];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = part[threadIdx.x] - s;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < count) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == kScanBlock - 1) tile_sums[blockIdx.x] = part[kScanBlock - 1];
}

__global__ __launch_bounds__(kScanBlock) void scan_add_kernel(int32_t* out, int64_t count,
                                                              const int32_t* tile_offsets) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  const int32_t add = tile_offsets[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < count) out[base + i] += add;
}

__global__ void scan_total_kernel(const int32_t* in, int32_t* out, int64_t count) {
  // out[count] = out[count-1] + in[count-1]
  if (count > 0) out[count] = out[count - 1] + in[count - 1];
  else out[0] = 0;
}

// ---------------------------------------------------------------- radix sort
__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__global__ __launch_bounds__(kWave) void radix_hist_kernel(const uint32_t* keys, int64_t count, int shift,
                                                           int64_t ntiles, int32_t* hist) {
  __shared__ int32_t h[kRadixBins];
  for (int d = threadIdx.x; d < kRadixBins; d += kWave) h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int r = 0; r < kRadixRounds; ++r) {
    const int64_t i = base + r * kWave + threadIdx.x;
    if (i < count) atomicAdd(&h[(keys[i] >> shift) & (kRadixBins - 1)], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadixBins; d += kWave) hist[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

// One wave per tile; keys are ranked stably inside each round of 64 by a ballot match on
// the digit bits, rounds are processed in order, so the scatter is a stable counting sort.
__global__ __launch_bounds__(kWave) void radix_scatter_kernel(const uint32_t* keys, const uint32_t* vals,
                                                              uint32_t* keys_out, uint32_t* vals_out,
                                                              int64_t count, int shift, int64_t ntiles,
                                                              const int32_t* offsets) {
  __shared__ int32_t base_off[kRadixBins];
  for (int d = threadIdx.x; d < kRadixBins; d += kWave)
    base_off[d] = offsets[(int64_t)d * ntiles + blockIdx.x];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  const uint64_t lt = lanemask_lt();
  for (int r = 0; r < kRadixRounds; ++r) {
    const int64_t i = base + r * kWave + threadIdx.x;
    const bool valid = i < count;
    uint32_t k = 0, v = 0;
    if (valid) {
      k = keys[i];
      v = vals[i];
    }
    const uint32_t d = (k >> shift) & (kRadixBins - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t mb = __ballot(bit);
      peers &= bit ? mb : ~mb;
    }
    const int rank = __popcll(peers & lt);
    const int cnt = __popcll(peers);
    int pos = 0;
    if (valid) pos = base_off[d] + rank;
    __syncthreads();
    if (valid) {
      keys_out[pos] = k;
      vals_out[pos] = v;
      if (rank == 0) base_off[d] += cnt;
    }
    __syncthreads();
  }
}

// Segment pointers from keys sorted ascending: ptr[c] = first position whose key is >= c.
// Thread i owns the boundary between positions i-1 and i and fills the pointers of every
// key value in (key[i-1], key[i]]; no atomics, so power-law heads cost nothing extra.
__global__ __launch_bounds__(256) void ptr_from_sorted_kernel(const uint32_t* keys, int64_t count, int64_t nseg,
                                                              int32_t* ptr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > count) return;
  const int64_t lo = (i == 0) ? 0 : (int64_t)keys[i - 1] + 1;
  const int64_t hi = (i == count) ? nseg : (int64_t)keys[i];
  for (int64_t c = lo; c <= hi; ++c) ptr[c] = (int32_t)i;
}

__global__ __launch_bounds__(256) void gather_csc_kernel(const uint32_t* perm, const int32_t* row_of,
                                                         const float* val, int64_t nnz, int32_t* row_csc,
                                                         float* val_csc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const uint32_t p = perm[i];
  row_csc[i] = row_of[p];
  val_csc[i] = val[p];
}

__global__ __launch_bounds__(256) void gather_values_kernel(const int32_t* perm, const float* val, int64_t nnz,
                                                            float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) out[i] = val[perm[i]];
}

// ---------------------------------------------------------------- merge-path tables
// Partition w starts on merge diagonal min(w*ipw, nseg+nnz) of the merge of the segment
// end offsets ptr[1..nseg] with the nonzero indices 0..nnz-1 (a segment end offset is
// taken before nonzero e when it is <= e).
__global__ __launch_bounds__(256) void merge_partition_kernel(const int32_t* ptr, int64_t nseg, int64_t nnz,
                                                              int64_t ipw, int64_t nwaves, int32_t* part_seg,
                                                              int32_t* part_e) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w > nwaves) return;
  const int64_t diag = min(w * ipw, nseg + nnz);
  int64_t lo = max(diag - nnz, (int64_t)0), hi = min(diag, nseg);
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)ptr[mid + 1] <= diag - mid - 1) lo = mid + 1;
    else hi = mid;
  }
  part_seg[w] = (int32_t)lo;
  part_e[w] = (int32_t)(diag - lo);
}

// For each wave w1 whose first segment c began in an earlier wave and ends inside w1,
// record the first wave w0 that carries a partial sum of c (waves w0..w1-1 all carry c).
__global__ __launch_bounds__(256) void merge_fixplan_kernel(const int32_t* ptr, int64_t nseg, int64_t nwaves,
                                                            const int32_t* part_seg, const int32_t* part_e,
                                                            int32_t* fix_w0) {
  const int64_t w1 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w1 >= nwaves) return;
  const int32_t c = part_seg[w1];
  int32_t w0 = -1;
  if (w1 > 0 && c < nseg && ptr[c] < part_e[w1] && c < part_seg[w1 + 1]) {
    int64_t w = w1 - 1;
    while (w > 0 && part_seg[w] == c) --w;
    w0 = (int32_t)w;
  }
  fix_w0[w1] = w0;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Row-blocked order of the transpose product, read off the column-major mirror (no second
// sort): the rows of a column ascend in the mirror, so the nonzeros of hot column h inside row
// block b are one contiguous run of that column, bounded by two binary searches. Segment
// b * H + h gets that run; tail segment nhs + t gets the whole of tail column tailcol[t]. The
// runs keep the mirror's order (rows ascending), the order a stable sort by (block, column)
// of the row-major positions gives.
__device__ __forceinline__ int32_t lower_row(const int32_t* rows, int32_t lo, int32_t hi, int64_t r) {
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if ((int64_t)rows[mid] < r) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void bcsc_hot_runs_kernel(const int32_t* cp, const int32_t* row_csc,
                                                            const int32_t* hotcol, int64_t hh, int64_t nblk,
                                                            int shift, int32_t* cnt, int32_t* src) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nblk * hh) return;
  const int64_t b = i / hh, h = i - b * hh;
  const int32_t c = hotcol[h];
  const int32_t lo = cp[c], hi = cp[c + 1];
  const int32_t s0 = lower_row(row_csc, lo, hi, b << shift);
  const int32_t s1 = lower_row(row_csc, s0, hi, (b + 1) << shift);
  cnt[i] = s1 - s0;
  src[i] = s0;
}

__global__ __launch_bounds__(256) void bcsc_tail_runs_kernel(const int32_t* cp, const int32_t* tailcol, int64_t ntail,
                                                             int64_t nhs, int32_t* cnt, int32_t* src) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= ntail) return;
  const int32_t c = tailcol[t];
  cnt[nhs + t] = cp[c + 1] - cp[c];
  src[nhs + t] = cp[c];
}

// A wave per segment copies its run of the mirror (rows, values, row-major positions).
// a wave per run; brow is null when only the values move
__global__ __launch_bounds__(256) void bcsc_copy_kernel(const int32_t* bptr, const int32_t* src, int64_t nseg,
                                                        const int32_t* row_csc, const float* val_csc,
                                                        int32_t* brow, float* bval) {
  const int64_t seg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (seg >= nseg) return;
  const int lane = threadIdx.x & 63;
  const int32_t d0 = bptr[seg], len = bptr[seg + 1] - d0, s0 = src[seg];
  for (int32_t i = lane; i < len; i += 64) {
    if (brow) brow[d0 + i] = row_csc[s0 + i];
    bval[d0 + i] = val_csc[s0 + i];
  }
}

}  // namespace

void launch_validate_csr(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                         const int32_t* col, const float* val, int* flag, hipStream_t st) {
  validate_rows_kernel<<<grid_for(m + 1, 256), 256, 0, st>>>(m, n, nnz, row_ptr, col, flag);
  if (nnz > 0) validate_vals_kernel<<<grid_for(nnz, 256), 256, 0, st>>>(nnz, val, flag);
}

void launch_ptr_to_i32(const int64_t* p, int64_t count, int32_t* out, hipStream_t st) {
  if (count > 0) ptr_to_i32_kernel<<<grid_for(count, 256), 256, 0, st>>>(p, count, out);
}

void launch_expand_rows(const int32_t* rp, int64_t m, int64_t nnz, int32_t* row_of, hipStream_t st) {
  if (nnz > 0) expand_rows_kernel<<<grid_for(nnz, 256), 256, 0, st>>>(rp, m, nnz, row_of);
}

size_t scan_temp_bytes(int64_t count) {
  size_t total = 0;
  int64_t c = count;
  while (c > 1) {
    const int64_t tiles = (c + kScanTile - 1) / kScanTile;
    total += 2 * (size_t)(tiles + 1) * sizeof(int32_t) + 256;
    c = tiles;
  }
  return total + 256;
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t count, void* temp, hipStream_t st) {
  if (count <= 0) {
    scan_total_kernel<<<1, 1, 0, st>>>(in, out, 0);
    return;
  }
  const int64_t tiles = (count + kScanTile - 1) / kScanTile;
  int32_t* sums = static_cast<int32_t*>(temp);
  int32_t* offs = sums + (tiles + 1);
  char* rest = reinterpret_cast<char*>(offs + (tiles + 1)) + 256;
  scan_tiles_kernel<<<(unsigned)tiles, kScanBlock, 0, st>>>(in, out, count, sums);
  if (tiles > 1) {
    exclusive_scan_i32(sums, offs, tiles, rest, st);
    scan_add_kernel<<<(unsigned)tiles, kScanBlock, 0, st>>>(out, count, offs);
  }
  scan_total_kernel<<<1, 1, 0, st>>>(in, out, count);
}

size_t radix_temp_bytes(int64_t count) {
  const int64_t ntiles = (count + kRadixTile - 1) / kRadixTile;
  const int64_t hn = ntiles * kRadixBins;
  return 2 * (size_t)(hn + 1) * sizeof(int32_t) + scan_temp_bytes(hn) + 512;
}

void radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                      int64_t count, int bits, void* temp, hipStream_t st) {
  if (count <= 0) return;
  const int64_t ntiles = (count + kRadixTile - 1) / kRadixTile;
  const int64_t hn = ntiles * kRadixBins;
  int32_t* hist = static_cast<int32_t*>(temp);
  int32_t* offs = hist + (hn + 1);
  void* scratch = offs + (hn + 1);
  scratch = reinterpret_cast<char*>(scratch) + 256;
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  uint32_t *ka = keys, *va = vals, *kb = keys_alt, *vb = vals_alt;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    radix_hist_kernel<<<(unsigned)ntiles, kWave, 0, st>>>(ka, count, shift, ntiles, hist);
    exclusive_scan_i32(hist, offs, hn, scratch, st);
    radix_scatter_kernel<<<(unsigned)ntiles, kWave, 0, st>>>(ka, va, kb, vb, count, shift, ntiles, offs);
    uint32_t* t = ka;
    ka = kb;
    kb = t;
    t = va;
    va = vb;
    vb = t;
  }
  if (ka != keys) {
    (void)hipMemcpyAsync(keys, ka, count * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(vals, va, count * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
  }
}

void launch_ptr_from_sorted(const uint32_t* keys, int64_t count, int64_t nseg, int32_t* ptr, hipStream_t st) {
  ptr_from_sorted_kernel<<<grid_for(count + 1, 256), 256, 0, st>>>(keys, count, nseg, ptr);
}

void launch_gather_csc(const uint32_t* perm, const int32_t* row_of, const float* val, int64_t nnz,
                       int32_t* row_csc, float* val_csc, hipStream_t st) {
  if (nnz > 0) gather_csc_kernel<<<grid_for(nnz, 256), 256, 0, st>>>(perm, row_of, val, nnz, row_csc, val_csc);
}

void launch_bcsc_runs(const int32_t* cp, const int32_t* row_csc, const int32_t* hotcol, const int32_t* tailcol,
                      int64_t hh, int64_t nblk, int64_t ntail, int shift, int32_t* cnt, int32_t* src, hipStream_t st) {
  const int64_t nhs = nblk * hh;
  if (nhs > 0)
    bcsc_hot_runs_kernel<<<grid_for(nhs, 256), 256, 0, st>>>(cp, row_csc, hotcol, hh, nblk, shift, cnt, src);
  if (ntail > 0) bcsc_tail_runs_kernel<<<grid_for(ntail, 256), 256, 0, st>>>(cp, tailcol, ntail, nhs, cnt, src);
}

void launch_bcsc_copy(const int32_t* bptr, const int32_t* src, int64_t nseg, const int32_t* row_csc,
                      const float* val_csc, int32_t* brow, float* bval, hipStream_t st) {
  if (nseg > 0)
    bcsc_copy_kernel<<<grid_for(nseg, 4), 256, 0, st>>>(bptr, src, nseg, row_csc, val_csc, brow, bval);
}

void launch_bcsc_values(const int32_t* bptr, const int32_t* src, int64_t nseg, const float* val_csc, float* bval,
                        hipStream_t st) {
  if (nseg > 0)
    bcsc_copy_kernel<<<grid_for(nseg, 4), 256, 0, st>>>(bptr, src, nseg, nullptr, val_csc, nullptr, bval);
}

void launch_gather_values(const int32_t* perm, const float* val, int64_t nnz, float* out, hipStream_t st) {
  if (nnz > 0) gather_values_kernel<<<grid_for(nnz, 256), 256, 0, st>>>(perm, val, nnz, out);
}

int64_t merge_items_per_wave(int64_t nseg, int64_t nnz) {
  // aim for >= 8192 partitions (32 waves per CU) with 128..2048 items each
  int64_t ipw = (nseg + nnz) / 8192;
  if (ipw < 128) ipw = 128;
  if (ipw > 2048) ipw = 2048;
  return ipw;
}

void launch_merge_partition(MergePlan& p, hipStream_t st) {
  merge_partition_kernel<<<grid_for(p.nwaves + 1, 256), 256, 0, st>>>(p.ptr, p.nseg, p.nnz, p.ipw, p.nwaves,
                                                                      p.part_seg, p.part_e);
}

void launch_merge_fixplan(MergePlan& p, hipStream_t st) {
  merge_fixplan_kernel<<<grid_for(p.nwaves, 256), 256, 0, st>>>(p.ptr, p.nseg, p.nwaves, p.part_seg, p.part_e,
                                                               p.fix_w0);
}

}  // namespace frpca
