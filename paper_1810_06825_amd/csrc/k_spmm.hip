// Sparse x tall-panel products of Alg. 5/6 (A Q and A^T Y), one kernel for both sides.
//
// The sparse operand is a "segment matrix": segment i lists (idx, val) pairs and the product
// is out[i, :] = sum val * in[idx, :]. CSR rows give A Q; the column-major mirror gives
// A^T Y, so the transpose product needs no atomics. Work is split by merge path (Merrill &
// Garland, SC'16): each wave owns an equal share of (nonzeros + segment ends), which keeps
// power-law columns with millions of entries balanced. A lane owns two panel columns
// (float2), so a wave streams one 2*64-wide panel row per nonzero; the (index, value)
// stream is read 64 entries per coalesced load and broadcast with readlane. Partial sums of segments cut by a partition
// boundary go to per-wave carry/head slots and a fix-up kernel adds them in wave order,
// so results are deterministic.
#include <climits>

#include "kernels.h"

namespace frpca {
namespace {

struct SpmmArgs {
  const int32_t* ptr;
  const int32_t* idx;
  const float* val;
  const int32_t* part_seg;
  const int32_t* part_e;
  int64_t nseg, nwaves;
  const void* in;
  int ld_in;
  float* out_f32;
  uint16_t* out_bf16;
  int ld_out;
  int lp;  // columns computed (even, <= 128)
  float* carry;
  float* head;
};

constexpr int kBatch = 8;  // gathers in flight per wave

// The sparse operand is read exactly once per product: non-temporal loads keep it from
// displacing the gathered panel rows in the caches.
template <class T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}

template <bool IN_BF16>
__global__ __launch_bounds__(256) void spmm_merge_kernel(SpmmArgs a) {
  const int lane = threadIdx.x & 63;
  // wave index made explicitly uniform so the partition bounds are scalar values
  const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= a.nwaves) return;
  const int col = 2 * lane;
  const bool act = col < a.lp;
  int seg = a.part_seg[w];
  const int seg_stop = a.part_seg[w + 1];
  int e = a.part_e[w];
  const int e_stop = a.part_e[w + 1];
  // the first segment continues a segment begun by an earlier wave
  bool pending_head = (seg < a.nseg) && (a.ptr[seg] < e);
  int next_end = (seg < seg_stop) ? a.ptr[seg + 1] : INT_MAX;
  float2 acc = make_float2(0.f, 0.f);

  auto emit = [&]() {
    if (act) {
      if (pending_head) {
        store2_f32(a.head, (size_t)w * 128 + col, acc);
      } else {
        const size_t o = (size_t)seg * a.ld_out + col;
        if (a.out_f32) store2_f32(a.out_f32, o, acc);
        if (a.out_bf16) store2_bf16(a.out_bf16, o, acc);
      }
    }
    pending_head = false;
    acc = make_float2(0.f, 0.f);
    ++seg;
    next_end = (seg < seg_stop) ? a.ptr[seg + 1] : INT_MAX;
  };

  // The (index, value) stream is read 64 entries at a time with one coalesced (streaming)
  // load per wave; entries are broadcast with readlane, the next window is in flight while
  // the current one is consumed.
  int wbase = e;
  int widx = 0, nidx = 0;
  float wval = 0.f, nval = 0.f;
  if (wbase + lane < e_stop) {
    widx = stream_load(a.idx + wbase + lane);
    wval = stream_load(a.val + wbase + lane);
  }
  while (e < e_stop) {
    const int wend = min(wbase + 64, e_stop);
    if (wbase + 64 + lane < e_stop) {
      nidx = stream_load(a.idx + wbase + 64 + lane);
      nval = stream_load(a.val + wbase + 64 + lane);
    }
    while (e < wend) {
      const int nb = min(kBatch, wend - e);
      const int off = e - wbase;
      int c[kBatch];
      float v[kBatch];
      float2 x[kBatch];
#pragma unroll
      for (int t = 0; t < kBatch; ++t) {
        if (t < nb) {
          c[t] = __builtin_amdgcn_readlane(widx, off + t);
          v[t] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wval), off + t));
        }
      }
#pragma unroll
      for (int t = 0; t < kBatch; ++t) {
        x[t] = make_float2(0.f, 0.f);
        if (t < nb && act) x[t] = load2<IN_BF16>(a.in, (size_t)c[t] * a.ld_in + col);
      }
#pragma unroll
      for (int t = 0; t < kBatch; ++t) {
        if (t < nb) {
          while (next_end <= e + t) emit();
          acc.x = fmaf(v[t], x[t].x, acc.x);
          acc.y = fmaf(v[t], x[t].y, acc.y);
        }
      }
      e += nb;
    }
    wbase += 64;
    widx = nidx;
    wval = nval;
  }
  while (seg < seg_stop) emit();
  if (seg_stop < a.nseg && act) store2_f32(a.carry, (size_t)w * 128 + col, acc);
}

// out[c] = carry[w0] + ... + carry[w1-1] + head[w1] for segments cut by partition bounds.
__global__ __launch_bounds__(256) void spmm_fixup_kernel(const int32_t* part_seg, const int32_t* fix_w0,
                                                         int64_t nwaves, const float* carry, const float* head,
                                                         float* out_f32, uint16_t* out_bf16, int ld_out, int lp) {
  const int lane = threadIdx.x & 63;
  const int64_t w1 = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w1 >= nwaves) return;
  const int w0 = fix_w0[w1];
  if (w0 < 0) return;
  const int col = 2 * lane;
  if (col >= lp) return;
  const int c = part_seg[w1];
  float2 s = make_float2(0.f, 0.f);
  for (int64_t w = w0; w < w1; ++w) {
    const float2 t = *reinterpret_cast<const float2*>(carry + (size_t)w * 128 + col);
    s.x += t.x;
    s.y += t.y;
  }
  const float2 h = *reinterpret_cast<const float2*>(head + (size_t)w1 * 128 + col);
  s.x += h.x;
  s.y += h.y;
  const size_t o = (size_t)c * ld_out + col;
  if (out_f32) store2_f32(out_f32, o, s);
  if (out_bf16) store2_bf16(out_bf16, o, s);
}

}  // namespace

void launch_spmm_main(const MergePlan& p, int lp, const void* in, bool in_bf16, int ld_in, float* out_f32,
                      uint16_t* out_bf16, int ld_out, hipStream_t st) {
  if (p.nwaves <= 0) return;
  SpmmArgs a{p.ptr, p.idx, p.val, p.part_seg, p.part_e, p.nseg, p.nwaves, in, ld_in, out_f32, out_bf16,
             ld_out, lp, p.carry, p.head};
  const unsigned grid = (unsigned)((p.nwaves + 3) / 4);
  if (in_bf16) spmm_merge_kernel<true><<<grid, 256, 0, st>>>(a);
  else spmm_merge_kernel<false><<<grid, 256, 0, st>>>(a);
}

void launch_spmm_fixup(const MergePlan& p, int lp, float* out_f32, uint16_t* out_bf16, int ld_out, hipStream_t st) {
  if (p.nwaves <= 0) return;
  const unsigned grid = (unsigned)((p.nwaves + 3) / 4);
  spmm_fixup_kernel<<<grid, 256, 0, st>>>(p.part_seg, p.fix_w0, p.nwaves, p.carry, p.head, out_f32, out_bf16,
                                          ld_out, lp);
}

void launch_spmm(const MergePlan& p, int lp, const void* in, bool in_bf16, int ld_in, float* out_f32,
                 uint16_t* out_bf16, int ld_out, hipStream_t st) {
  launch_spmm_main(p, lp, in, in_bf16, ld_in, out_f32, out_bf16, ld_out, st);
  launch_spmm_fixup(p, lp, out_f32, out_bf16, ld_out, st);
}

}  // namespace frpca
