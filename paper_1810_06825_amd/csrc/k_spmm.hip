// Sparse x tall-panel products of Alg. 5/6 (A Q and A^T Y), one kernel for both sides.
//
// The sparse operand is a "segment matrix": segment i lists (idx, val) pairs and the product
// is out[i, :] = sum val * in[idx, :]. CSR rows give A Q; the column-major mirror gives
// A^T Y, so the transpose product needs no atomics. Work is split by merge path (Merrill &
// Garland, SC'16): each wave owns an equal share of (nonzeros + segment ends), which keeps
// power-law columns with millions of entries balanced. The (index, value) stream is read 64
// entries per coalesced load and broadcast with readlane. In the basic form a lane owns two
// panel columns (float2), so a wave gathers one panel row per nonzero; panels whose rows
// are 16-byte aligned with a computed width that is a multiple of 4 take the paired form
// further down, where one 16-byte load per lane fetches two panel rows. Partial sums of
// segments cut by a partition boundary go to per-wave carry/head slots and a fix-up kernel
// adds them in wave order, so results are deterministic.
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
  int sweep;
  const int32_t* out_row;  // output row of each segment (identity when null)
  const float* csub_v;     // rank-1 term out[r] -= csub_s[r] * csub_v (none when null)
  const float* csub_s;     //   (factor 1 when null)
  int32_t* sweep_ctr;      // sweep mode: per-XCD partition tickets (zeroed before each launch)
};

// Sweep mode: a grid of resident waves takes the partitions from counters. The partitions are
// dealt to the XCDs in chunks of kSweepChunk consecutive ones (chunk j to XCD j mod 8, by the
// hardware's round-robin placement of blocks on XCDs), and the waves of an XCD take its
// partitions in order, each wave its next one from the XCD's counter when it finishes the last.
// The partitions in flight on an XCD then stay within about one chunk of the segment order,
// which the row-blocked transpose product needs for its gathered panel rows to stay in that
// XCD's L2. (Walking fixed rounds instead let the waves drift apart over the rounds and widened
// the band: the hot part of the 12.9M-row transpose product took 6.2 ms against 4.2.)
#ifndef FRPCA_SWEEP_CHUNK
#define FRPCA_SWEEP_CHUNK 512
#endif
constexpr int kSweepChunk = FRPCA_SWEEP_CHUNK;

template <class F>
__device__ __forceinline__ void sweep_partitions(const SpmmArgs& a, int lane, F&& run) {
  const int nx = min((int)gridDim.x, 8);  // virtual XCDs, each with at least one block
  const int x = blockIdx.x % nx;
  int* ctr = a.sweep_ctr + 32 * x;  // one counter per 128-byte line
  int t = 0;
  if (lane == 0) t = atomicAdd(ctr, 1);
  int k = __builtin_amdgcn_readlane(t, 0);
  for (;;) {
    // the XCD's k-th partition: tickets are handed out in increasing order and this map is
    // increasing in k, so once a ticket lies past the end every later one does too
    const int64_t w = ((int64_t)(k / kSweepChunk) * nx + x) * kSweepChunk + k % kSweepChunk;
    if (w >= a.nwaves) break;
    if (lane == 0) t = atomicAdd(ctr, 1);  // the next ticket, taken before this partition's work
    run(w);
    k = __builtin_amdgcn_readlane(t, 0);
  }
}

__global__ void sweep_reset_kernel(int32_t* ctr) { ctr[threadIdx.x] = 0; }

constexpr int kBatch = 8;  // gathers in flight per wave
#ifndef FRPCA_SWEEP_BLOCKS
#define FRPCA_SWEEP_BLOCKS 1024
#endif
// resident blocks of 4 waves in sweep mode (4 per CU): a narrower band of row blocks in flight
// keeps more of the gathered rows in L2 (1024 measured best against 512 to 2048)
constexpr unsigned kSweepBlocks = FRPCA_SWEEP_BLOCKS;

// The sparse operand is read exactly once per product: non-temporal loads keep it from
// displacing the gathered panel rows in the caches.
template <class T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}

template <bool IN_BF16>
__device__ __forceinline__ void spmm_partition(const SpmmArgs& a, int64_t w, int lane, int* lw) {
  const int col = 2 * lane;
  const bool act = col < a.lp;
  int seg = a.part_seg[w];
  const int seg_stop = a.part_seg[w + 1];
  int e = a.part_e[w];
  const int e_stop = a.part_e[w + 1];
  // the first segment continues a segment begun by an earlier wave
  bool pending_head = (seg < a.nseg) && (a.ptr[seg] < e);
  // segment ends (and output rows) come 64 at a time in one coalesced load, parked in the
  // wave's LDS window and read from there: a global load at every segment end would wait for
  // all gathers in flight (the window's own refill waits once per 64 segments)
  int pbase = seg;
  auto refill = [&]() {
    lw[lane] = (pbase + 1 + lane <= a.nseg) ? a.ptr[pbase + 1 + lane] : INT_MAX;
    if (a.out_row) lw[64 + lane] = (pbase + lane < a.nseg) ? a.out_row[pbase + lane] : 0;
  };
  refill();
  int next_end = (seg < seg_stop) ? __builtin_amdgcn_readfirstlane(lw[0]) : INT_MAX;
  float2 acc = make_float2(0.f, 0.f);

  auto emit = [&]() {
    if (act) {
      if (pending_head) {
        store2_f32(a.head, (size_t)w * 128 + col, acc);
      } else {
        const int64_t orow = a.out_row ? lw[64 + seg - pbase] : seg;
        float2 t = acc;
        if (a.csub_v) {
          const float sc = a.csub_s ? a.csub_s[orow] : 1.f;
          t.x -= sc * a.csub_v[col];
          t.y -= sc * a.csub_v[col + 1];
        }
        const size_t o = (size_t)orow * a.ld_out + col;
        if (a.out_f32) store2_f32(a.out_f32, o, t);
        if (a.out_bf16) store2_bf16(a.out_bf16, o, t);
      }
    }
    pending_head = false;
    acc = make_float2(0.f, 0.f);
    ++seg;
    if (seg < seg_stop) {
      if (seg - pbase >= 64) {
        pbase += 64;
        refill();
      }
      next_end = __builtin_amdgcn_readfirstlane(lw[seg - pbase]);
    } else {
      next_end = INT_MAX;
    }
  };

  // The (index, value) stream is read 64 entries at a time with one coalesced (streaming)
  // load per wave; entries are broadcast with readlane, the next window is in flight while
  // the current one is consumed. Gathers run as a two-stage pipeline: batch j+1's panel rows
  // are requested before batch j's are accumulated, so up to 2 kBatch rows are in flight per
  // wave. Lanes past lp gather column 0 (in bounds, never stored) instead of branching.
  const int gcol = act ? col : 0;
  int wbase = e;
  int widx = 0, nidx = 0;
  float wval = 0.f, nval = 0.f;
  if (wbase + lane < e_stop) {
    widx = stream_load(a.idx + wbase + lane);
    wval = stream_load(a.val + wbase + lane);
  }
  float pv[kBatch];
  float2 px[kBatch];
  int pe = 0, pnb = 0;  // pending batch: first entry and size (0: none)
  auto consume = [&]() {
#pragma unroll
    for (int t = 0; t < kBatch; ++t) {
      if (t < pnb) {
        while (next_end <= pe + t) emit();
        acc.x = fmaf(pv[t], px[t].x, acc.x);
        acc.y = fmaf(pv[t], px[t].y, acc.y);
      }
    }
  };
  while (e < e_stop) {
    const int wend = min(wbase + 64, e_stop);
    if (wbase + 64 + lane < e_stop) {
      nidx = stream_load(a.idx + wbase + 64 + lane);
      nval = stream_load(a.val + wbase + 64 + lane);
    }
    while (e < wend) {
      const int nb = min(kBatch, wend - e);
      const int off = e - wbase;
      float v[kBatch];
      float2 x[kBatch];
      if (nb == kBatch) {
#pragma unroll
        for (int t = 0; t < kBatch; ++t) {
          const int c = __builtin_amdgcn_readlane(widx, off + t);
          v[t] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wval), off + t));
          x[t] = load2<IN_BF16>(a.in, (size_t)c * a.ld_in + gcol);
        }
      } else {
#pragma unroll
        for (int t = 0; t < kBatch; ++t) {
          v[t] = 0.f;
          x[t] = make_float2(0.f, 0.f);
          if (t < nb) {
            const int c = __builtin_amdgcn_readlane(widx, off + t);
            v[t] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wval), off + t));
            x[t] = load2<IN_BF16>(a.in, (size_t)c * a.ld_in + gcol);
          }
        }
      }
      consume();
#pragma unroll
      for (int t = 0; t < kBatch; ++t) {
        pv[t] = v[t];
        px[t] = x[t];
      }
      pe = e;
      pnb = nb;
      e += nb;
    }
    wbase += 64;
    widx = nidx;
    wval = nval;
  }
  consume();
  while (seg < seg_stop) emit();
  if (seg_stop < a.nseg && act) store2_f32(a.carry, (size_t)w * 128 + col, acc);
}

template <bool IN_BF16>
__global__ __launch_bounds__(256) void spmm_merge_kernel(SpmmArgs a) {
  __shared__ int win[4][128];  // per wave: 64 segment ends, then 64 output rows
  const int lane = threadIdx.x & 63;
  // wave index made explicitly uniform so the partition bounds are scalar values
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int* lw = win[wv];
  if (!a.sweep) {
    const int64_t w = (int64_t)blockIdx.x * 4 + wv;
    if (w < a.nwaves) spmm_partition<IN_BF16>(a, w, lane, lw);
    return;
  }
  sweep_partitions(a, lane, [&](int64_t w) { spmm_partition<IN_BF16>(a, w, lane, lw); });
}

// ---------------------------------------------------------------------------------------
// Paired gathers (panels of 4-aligned width): vector-memory instructions, not bytes, bound
// the products above (each one costs the texture addresser the same cycles whatever its
// width), so a 16-byte load per lane lets one instruction fetch two panel rows: lanes 0-31
// take the even entry of each pair of nonzeros, lanes 32-63 the odd one, a lane covering four
// columns. The halves accumulate separately and are added with a cross-half shuffle when a
// segment ends; a segment ending between the two entries of a pair is handled by letting
// only the even half accumulate, emitting, then adding the odd half.
#ifndef FRPCA_SPMM_PAIRS
#define FRPCA_SPMM_PAIRS 4
#endif
constexpr int kPairs = FRPCA_SPMM_PAIRS;  // pairs per batch; two batches in flight
#ifndef FRPCA_SPMM_NT_STORE
#define FRPCA_SPMM_NT_STORE 1
#endif

// NT: streaming (non-temporal) gathers, for panels so much larger than the Infinity Cache
// that a gathered row is almost never found there again
template <bool IN_BF16, bool NT>
__device__ __forceinline__ float4 load4(const void* base, size_t idx) {
  if constexpr (IN_BF16) {
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    const v2u* q = reinterpret_cast<const v2u*>(static_cast<const uint16_t*>(base) + idx);
    v2u w;
    if constexpr (NT) w = __builtin_nontemporal_load(q);
    else w = *q;
    return make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u), __uint_as_float(w.y << 16),
                       __uint_as_float(w.y & 0xFFFF0000u));
  } else {
    if constexpr (NT) {
      typedef float v4f __attribute__((ext_vector_type(4)));
      const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(static_cast<const float*>(base) + idx));
      return make_float4(t.x, t.y, t.z, t.w);
    } else {
      return *reinterpret_cast<const float4*>(static_cast<const float*>(base) + idx);
    }
  }
}

__device__ __forceinline__ void fma4(float4& acc, float v, const float4& x) {
  acc.x = fmaf(v, x.x, acc.x);
  acc.y = fmaf(v, x.y, acc.y);
  acc.z = fmaf(v, x.z, acc.z);
  acc.w = fmaf(v, x.w, acc.w);
}

template <bool IN_BF16, bool NT>
__device__ __forceinline__ void spmm_partition4(const SpmmArgs& a, int64_t w, int lane, int* lw) {
  const int half = lane >> 5;
  const int col = 4 * (lane & 31);
  const bool act = col < a.lp;
  const int gcol = act ? col : 0;
  int seg = a.part_seg[w];
  const int seg_stop = a.part_seg[w + 1];
  int e = a.part_e[w];
  const int e_stop = a.part_e[w + 1];
  bool pending_head = (seg < a.nseg) && (a.ptr[seg] < e);
  // segment ends (and output rows) come 64 at a time in one coalesced load, parked in the
  // wave's LDS window and read from there: a global load at every segment end would wait for
  // all gathers in flight (the window's own refill waits once per 64 segments)
  int pbase = seg;
  auto refill = [&]() {
    lw[lane] = (pbase + 1 + lane <= a.nseg) ? a.ptr[pbase + 1 + lane] : INT_MAX;
    if (a.out_row) lw[64 + lane] = (pbase + lane < a.nseg) ? a.out_row[pbase + lane] : 0;
  };
  refill();
  int next_end = (seg < seg_stop) ? __builtin_amdgcn_readfirstlane(lw[0]) : INT_MAX;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);

  auto emit = [&]() {
    float4 t;
    t.x = acc.x + __shfl_xor(acc.x, 32);
    t.y = acc.y + __shfl_xor(acc.y, 32);
    t.z = acc.z + __shfl_xor(acc.z, 32);
    t.w = acc.w + __shfl_xor(acc.w, 32);
    if (half == 0 && act) {
      if (pending_head) {
        *reinterpret_cast<float4*>(a.head + (size_t)w * 128 + col) = t;
      } else {
        const int64_t orow = a.out_row ? lw[64 + seg - pbase] : seg;
        if (a.csub_v) {
          const float sc = a.csub_s ? a.csub_s[orow] : 1.f;
          const float4 cv = *reinterpret_cast<const float4*>(a.csub_v + col);
          t.x -= sc * cv.x;
          t.y -= sc * cv.y;
          t.z -= sc * cv.z;
          t.w -= sc * cv.w;
        }
        const size_t o = (size_t)orow * a.ld_out + col;
#if FRPCA_SPMM_NT_STORE
        // streaming stores: output rows are not read again by this launch, so they should not
        // displace gathered panel rows from L2
        typedef float v4f __attribute__((ext_vector_type(4)));
        if (a.out_f32) {
          const v4f tv = {t.x, t.y, t.z, t.w};
          __builtin_nontemporal_store(tv, reinterpret_cast<v4f*>(a.out_f32 + o));
        }
#else
        if (a.out_f32) *reinterpret_cast<float4*>(a.out_f32 + o) = t;
#endif
        if (a.out_bf16) {
          uint2 b;
          b.x = (uint32_t)f32_to_bf16(t.x) | ((uint32_t)f32_to_bf16(t.y) << 16);
          b.y = (uint32_t)f32_to_bf16(t.z) | ((uint32_t)f32_to_bf16(t.w) << 16);
          *reinterpret_cast<uint2*>(a.out_bf16 + o) = b;
        }
      }
    }
    pending_head = false;
    acc = make_float4(0.f, 0.f, 0.f, 0.f);
    ++seg;
    if (seg < seg_stop) {
      if (seg - pbase >= 64) {
        pbase += 64;
        refill();
      }
      next_end = __builtin_amdgcn_readfirstlane(lw[seg - pbase]);
    } else {
      next_end = INT_MAX;
    }
  };

  int wbase = e;
  int widx = 0, nidx = 0;
  float wval = 0.f, nval = 0.f;
  if (wbase + lane < e_stop) {
    widx = stream_load(a.idx + wbase + lane);
    wval = stream_load(a.val + wbase + lane);
  }
  float pv[kPairs];
  float4 px[kPairs];
  int pe = 0, pend = 0;  // pending batch: entries [pe, pend)
  auto consume = [&]() {
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      const int ep = pe + 2 * p;
      if (ep < pend) {
        while (next_end <= ep) emit();
        if (ep + 1 < pend && next_end == ep + 1) {
          fma4(acc, half == 0 ? pv[p] : 0.f, px[p]);
          while (next_end <= ep + 1) emit();
          fma4(acc, half == 1 ? pv[p] : 0.f, px[p]);
        } else {
          fma4(acc, pv[p], px[p]);
        }
      }
    }
  };
  while (e < e_stop) {
    const int wend = min(wbase + 64, e_stop);
    if (wbase + 64 + lane < e_stop) {
      nidx = stream_load(a.idx + wbase + 64 + lane);
      nval = stream_load(a.val + wbase + 64 + lane);
    }
    while (e < wend) {
      const int stop = min(e + 2 * kPairs, wend);
      const int off = e - wbase;
      float v[kPairs];
      float4 x[kPairs];
#pragma unroll
      for (int p = 0; p < kPairs; ++p) {
        // this half's entry of pair p (entries past the batch gather row 0 with weight 0)
        const int src = off + 2 * p + half;
        const bool valid = e + 2 * p + half < stop;
        const int c = __shfl(widx, src & 63);
        const float vv = __shfl(wval, src & 63);
        v[p] = valid ? vv : 0.f;
        x[p] = load4<IN_BF16, NT>(a.in, (size_t)(valid ? c : 0) * a.ld_in + gcol);
      }
      consume();
#pragma unroll
      for (int p = 0; p < kPairs; ++p) {
        pv[p] = v[p];
        px[p] = x[p];
      }
      pe = e;
      pend = stop;
      e = stop;
    }
    wbase += 64;
    widx = nidx;
    wval = nval;
  }
  consume();
  while (seg < seg_stop) emit();
  if (seg_stop < a.nseg) {
    const float4 t = make_float4(acc.x + __shfl_xor(acc.x, 32), acc.y + __shfl_xor(acc.y, 32),
                                 acc.z + __shfl_xor(acc.z, 32), acc.w + __shfl_xor(acc.w, 32));
    if (half == 0 && act) *reinterpret_cast<float4*>(a.carry + (size_t)w * 128 + col) = t;
  }
}

#ifndef FRPCA_SPMM_QUAD
#define FRPCA_SPMM_QUAD 1
#endif
#ifndef FRPCA_SPMM_MINW
#define FRPCA_SPMM_MINW 1
#endif
template <bool IN_BF16, bool NT>
__global__ __launch_bounds__(256, FRPCA_SPMM_MINW) void spmm_merge4_kernel(SpmmArgs a) {
  __shared__ int win[4][128];  // per wave: 64 segment ends, then 64 output rows
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int* lw = win[wv];
  if (!a.sweep) {
    const int64_t w = (int64_t)blockIdx.x * 4 + wv;
    if (w < a.nwaves) spmm_partition4<IN_BF16, NT>(a, w, lane, lw);
    return;
  }
  sweep_partitions(a, lane, [&](int64_t w) { spmm_partition4<IN_BF16, NT>(a, w, lane, lw); });
}

// ---------------------------------------------------------------------------------------
// Quad gathers, for panels of at most 64 computed columns (where the paired kernel would
// leave half of each half-wave idle): the lanes of quarter q (lane / 16) take entry 4i + q of
// each quad of nonzeros, sixteen lanes covering 64 columns at four per lane, so one
// vector-memory instruction still fetches four rows. The quarters meet through two
// cross-quarter shuffles at each segment end; a segment ending inside a quad takes the
// quarters before its end.
constexpr int kQuads = 4;  // quads per batch; two batches in flight

template <bool IN_BF16, bool NT>
__device__ __forceinline__ void spmm_partition_q(const SpmmArgs& a, int64_t w, int lane, int* lw) {
  const int quarter = lane >> 4;
  const int col = 4 * (lane & 15);
  const bool act = col < a.lp;
  const int gcol = act ? col : 0;
  int seg = a.part_seg[w];
  const int seg_stop = a.part_seg[w + 1];
  int e = a.part_e[w];
  const int e_stop = a.part_e[w + 1];
  bool pending_head = (seg < a.nseg) && (a.ptr[seg] < e);
  int pbase = seg;
  auto refill = [&]() {
    lw[lane] = (pbase + 1 + lane <= a.nseg) ? a.ptr[pbase + 1 + lane] : INT_MAX;
    if (a.out_row) lw[64 + lane] = (pbase + lane < a.nseg) ? a.out_row[pbase + lane] : 0;
  };
  refill();
  int next_end = (seg < seg_stop) ? __builtin_amdgcn_readfirstlane(lw[0]) : INT_MAX;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);

  auto quad_sum = [&]() {
    float4 t;
    t.x = acc.x + __shfl_xor(acc.x, 16);
    t.y = acc.y + __shfl_xor(acc.y, 16);
    t.z = acc.z + __shfl_xor(acc.z, 16);
    t.w = acc.w + __shfl_xor(acc.w, 16);
    t.x += __shfl_xor(t.x, 32);
    t.y += __shfl_xor(t.y, 32);
    t.z += __shfl_xor(t.z, 32);
    t.w += __shfl_xor(t.w, 32);
    return t;
  };
  auto emit = [&]() {
    float4 t = quad_sum();
    if (quarter == 0 && act) {
      if (pending_head) {
        *reinterpret_cast<float4*>(a.head + (size_t)w * 128 + col) = t;
      } else {
        const int64_t orow = a.out_row ? lw[64 + seg - pbase] : seg;
        if (a.csub_v) {
          const float sc = a.csub_s ? a.csub_s[orow] : 1.f;
          const float4 cv = *reinterpret_cast<const float4*>(a.csub_v + col);
          t.x -= sc * cv.x;
          t.y -= sc * cv.y;
          t.z -= sc * cv.z;
          t.w -= sc * cv.w;
        }
        const size_t o = (size_t)orow * a.ld_out + col;
        typedef float v4f __attribute__((ext_vector_type(4)));
        if (a.out_f32) {
          const v4f tv = {t.x, t.y, t.z, t.w};
          __builtin_nontemporal_store(tv, reinterpret_cast<v4f*>(a.out_f32 + o));
        }
        if (a.out_bf16) {
          uint2 b;
          b.x = (uint32_t)f32_to_bf16(t.x) | ((uint32_t)f32_to_bf16(t.y) << 16);
          b.y = (uint32_t)f32_to_bf16(t.z) | ((uint32_t)f32_to_bf16(t.w) << 16);
          *reinterpret_cast<uint2*>(a.out_bf16 + o) = b;
        }
      }
    }
    pending_head = false;
    acc = make_float4(0.f, 0.f, 0.f, 0.f);
    ++seg;
    if (seg < seg_stop) {
      if (seg - pbase >= 64) {
        pbase += 64;
        refill();
      }
      next_end = __builtin_amdgcn_readfirstlane(lw[seg - pbase]);
    } else {
      next_end = INT_MAX;
    }
  };

  int wbase = e;
  int widx = 0, nidx = 0;
  float wval = 0.f, nval = 0.f;
  if (wbase + lane < e_stop) {
    widx = stream_load(a.idx + wbase + lane);
    wval = stream_load(a.val + wbase + lane);
  }
  float pv[kQuads];
  float4 px[kQuads];
  int pe = 0, pend = 0;  // pending batch: entries [pe, pend)
  auto consume = [&]() {
#pragma unroll
    for (int p = 0; p < kQuads; ++p) {
      const int eq = pe + 4 * p;
      if (eq < pend) {
        while (next_end <= eq) emit();
        // quarters lo.. of the quad are still to be added; a segment that ends after entry
        // next_end - 1 inside the quad takes the quarters before its end
        int lo = 0;
        while (next_end < eq + 4 && next_end < pend) {
          const int hi = next_end - eq;
          fma4(acc, (quarter >= lo && quarter < hi) ? pv[p] : 0.f, px[p]);
          lo = hi;
          while (next_end <= eq + lo) emit();
        }
        fma4(acc, quarter >= lo ? pv[p] : 0.f, px[p]);
      }
    }
  };
  while (e < e_stop) {
    const int wend = min(wbase + 64, e_stop);
    if (wbase + 64 + lane < e_stop) {
      nidx = stream_load(a.idx + wbase + 64 + lane);
      nval = stream_load(a.val + wbase + 64 + lane);
    }
    while (e < wend) {
      const int stop = min(e + 4 * kQuads, wend);
      const int off = e - wbase;
      float v[kQuads];
      float4 x[kQuads];
#pragma unroll
      for (int p = 0; p < kQuads; ++p) {
        // this quarter's entry of quad p (entries past the batch gather row 0 with weight 0)
        const int src = off + 4 * p + quarter;
        const bool valid = e + 4 * p + quarter < stop;
        const int c = __shfl(widx, src & 63);
        const float vv = __shfl(wval, src & 63);
        v[p] = valid ? vv : 0.f;
        x[p] = load4<IN_BF16, NT>(a.in, (size_t)(valid ? c : 0) * a.ld_in + gcol);
      }
      consume();
#pragma unroll
      for (int p = 0; p < kQuads; ++p) {
        pv[p] = v[p];
        px[p] = x[p];
      }
      pe = e;
      pend = stop;
      e = stop;
    }
    wbase += 64;
    widx = nidx;
    wval = nval;
  }
  consume();
  while (seg < seg_stop) emit();
  if (seg_stop < a.nseg) {
    const float4 t = quad_sum();
    if (quarter == 0 && act) *reinterpret_cast<float4*>(a.carry + (size_t)w * 128 + col) = t;
  }
}

template <bool IN_BF16, bool NT>
__global__ __launch_bounds__(256, FRPCA_SPMM_MINW) void spmm_quad_kernel(SpmmArgs a) {
  __shared__ int win[4][128];  // per wave: 64 segment ends, then 64 output rows
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int* lw = win[wv];
  if (!a.sweep) {
    const int64_t w = (int64_t)blockIdx.x * 4 + wv;
    if (w < a.nwaves) spmm_partition_q<IN_BF16, NT>(a, w, lane, lw);
    return;
  }
  sweep_partitions(a, lane, [&](int64_t w) { spmm_partition_q<IN_BF16, NT>(a, w, lane, lw); });
}

// out[c] = carry[w0] + ... + carry[w1-1] + head[w1] for segments cut by partition bounds
// (row c of out, or row out_row[c] when the plan maps segments to output rows). A wave takes
// kFixPerWave consecutive partitions (one launch-sized block per partition was bound by block
// dispatch, most partitions ending a single cut row).
constexpr int kFixPerWave = 8;
__global__ __launch_bounds__(256) void spmm_fixup_kernel(const int32_t* __restrict__ part_seg,
                                                         const int32_t* __restrict__ fix_w0, int64_t nwaves,
                                                         const float* __restrict__ carry,
                                                         const float* __restrict__ head, float* __restrict__ out_f32,
                                                         uint16_t* __restrict__ out_bf16, int ld_out, int lp,
                                                         const int32_t* __restrict__ out_row,
                                                         const float* __restrict__ csub_v,
                                                         const float* __restrict__ csub_s) {
  const int lane = threadIdx.x & 63;
  const int col = 2 * lane;
  if (col >= lp) return;
  const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wbeg = wave * kFixPerWave;
  // the partitions' bounds first, so their loads are in flight together
  int w0s[kFixPerWave], cs[kFixPerWave];
#pragma unroll
  for (int k = 0; k < kFixPerWave; ++k) {
    const bool in = wbeg + k < nwaves;
    w0s[k] = in ? fix_w0[wbeg + k] : -1;
    cs[k] = in ? part_seg[wbeg + k] : 0;
  }
#pragma unroll
  for (int k = 0; k < kFixPerWave; ++k) {
    const int64_t w1 = wbeg + k;
    const int w0 = w0s[k];
    if (w0 < 0) continue;
    const float2 h = *reinterpret_cast<const float2*>(head + (size_t)w1 * 128 + col);
    float2 s = make_float2(0.f, 0.f);
    for (int64_t w = w0; w < w1; ++w) {
      const float2 t = *reinterpret_cast<const float2*>(carry + (size_t)w * 128 + col);
      s.x += t.x;
      s.y += t.y;
    }
    s.x += h.x;
    s.y += h.y;
    const int c = cs[k];
    const int64_t orow = out_row ? out_row[c] : c;
    if (csub_v) {
      const float sc = csub_s ? csub_s[orow] : 1.f;
      s.x -= sc * csub_v[col];
      s.y -= sc * csub_v[col + 1];
    }
    const size_t o = (size_t)orow * ld_out + col;
    if (out_f32) store2_f32(out_f32, o, s);
    if (out_bf16) store2_bf16(out_bf16, o, s);
  }
}

}  // namespace

void launch_spmm_main(const MergePlan& p, int lp, const void* in, bool in_bf16, int ld_in, float* out_f32,
                      uint16_t* out_bf16, int ld_out, hipStream_t st, SpmmCorr corr) {
  if (p.nwaves <= 0) return;
  SpmmArgs a{p.ptr, p.idx, p.val, p.part_seg, p.part_e, p.nseg, p.nwaves, in, ld_in, out_f32, out_bf16,
             ld_out, lp, p.carry, p.head, p.sweep, p.out_row, corr.v, corr.s, p.sweep_ctr};
  if (p.sweep) sweep_reset_kernel<<<1, 256, 0, st>>>(p.sweep_ctr);  // a kernel, not a memset: capturable
  unsigned grid = (unsigned)((p.nwaves + 3) / 4);
  if (p.sweep && grid > kSweepBlocks) grid = kSweepBlocks;
  // paired 16-byte gathers when every row of in and out starts 16-byte (FP32) or 8-byte
  // (BF16) aligned and the computed width is a multiple of 4
  const size_t ein = in_bf16 ? 2 : 4;
  const bool al_in = (reinterpret_cast<uintptr_t>(in) % (4 * ein)) == 0 && (ld_in % 4) == 0;
  const bool al_out = (!out_f32 || (reinterpret_cast<uintptr_t>(out_f32) % 16) == 0) &&
                      (!out_bf16 || (reinterpret_cast<uintptr_t>(out_bf16) % 8) == 0) && (ld_out % 4) == 0;
  if ((lp % 4) == 0 && al_in && al_out) {
    // streaming gathers for a panel many times the Infinity Cache (not in sweep mode, whose
    // gathered rows are meant to stay in L2)
    const bool nt = !p.sweep && p.in_rows > 0 && (double)p.in_rows * ld_in * ein > kStreamPanelBytes;
    if (lp <= 64 && FRPCA_SPMM_QUAD) {
      if (in_bf16) {
        if (nt) spmm_quad_kernel<true, true><<<grid, 256, 0, st>>>(a);
        else spmm_quad_kernel<true, false><<<grid, 256, 0, st>>>(a);
      } else {
        if (nt) spmm_quad_kernel<false, true><<<grid, 256, 0, st>>>(a);
        else spmm_quad_kernel<false, false><<<grid, 256, 0, st>>>(a);
      }
      return;
    }
    if (in_bf16) {
      if (nt) spmm_merge4_kernel<true, true><<<grid, 256, 0, st>>>(a);
      else spmm_merge4_kernel<true, false><<<grid, 256, 0, st>>>(a);
    } else {
      if (nt) spmm_merge4_kernel<false, true><<<grid, 256, 0, st>>>(a);
      else spmm_merge4_kernel<false, false><<<grid, 256, 0, st>>>(a);
    }
    return;
  }
  if (in_bf16) spmm_merge_kernel<true><<<grid, 256, 0, st>>>(a);
  else spmm_merge_kernel<false><<<grid, 256, 0, st>>>(a);
}

void launch_spmm_fixup(const MergePlan& p, int lp, float* out_f32, uint16_t* out_bf16, int ld_out, hipStream_t st,
                       SpmmCorr corr) {
  if (p.nwaves <= 0) return;
  const int64_t fwaves = (p.nwaves + kFixPerWave - 1) / kFixPerWave;
  const unsigned grid = (unsigned)((fwaves + 3) / 4);
  spmm_fixup_kernel<<<grid, 256, 0, st>>>(p.part_seg, p.fix_w0, p.nwaves, p.carry, p.head, out_f32, out_bf16,
                                          ld_out, lp, p.out_row, corr.v, corr.s);
}

void launch_spmm(const MergePlan& p, int lp, const void* in, bool in_bf16, int ld_in, float* out_f32,
                 uint16_t* out_bf16, int ld_out, hipStream_t st, SpmmCorr corr) {
  launch_spmm_main(p, lp, in, in_bf16, ld_in, out_f32, out_bf16, ld_out, st, corr);
  launch_spmm_fixup(p, lp, out_f32, out_bf16, ld_out, st, corr);
}

}  // namespace frpca
