// LU basis of Lemma 3 / eq. (8): Q = P^T L for P X = L U, i.e. Q = X U^-1.
//
// Pivot rows are chosen by tournament pivoting (Grigori, Demmel & Xiang, "CALU", SIMAX
// 2011): leaves of 512 rows each run Gaussian elimination with partial pivoting (GEPP), one
// row per thread held in registers, and keep the <= l rows they pivot on; groups of four
// candidate sets (4 l <= 512 rows) are merged by GEPP again until one set remains. The
// root's GEPP fixes the pivot order and which columns have a usable pivot (best remaining
// |entry| > tol * max|X|; inner nodes only skip exactly-zero columns). A final kernel factors
// the pivot rows (no further pivoting needed) in FP64, inverts U in place and scatters U^-1
// into an l x l coefficient matrix B (zero rows/columns for columns without a pivot), so
// Q = X B runs on the MFMA panel kernel. Any pivot choice gives a P^T L spanning range(X)
// (Lemma 3); the pivot rows of Q form a unit lower-triangular block.
#include <type_traits>

#include "kernels.h"

namespace frpca {
namespace {

constexpr int kNode = 512;   // rows per tournament node (one per thread)
constexpr int kFanIn = 4;    // candidate sets merged per node (4 * 128 <= 512)
constexpr int kWaves = kNode / 64;
static_assert(kNode <= 512, "the argmax key keeps 9 bits for the row slot");

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Largest 32-bit key of the wave: DPP row shifts 1, 2, 4, 8 (lane 15 of each row of 16 then
// holds its row's maximum; lanes whose source falls outside the row keep their own key), then
// the four row maxima through readlane. Every lane gets the result. All 64 lanes must be active.
__device__ __forceinline__ uint32_t wave_max_key(uint32_t k) {
  k = max(k, (uint32_t)__builtin_amdgcn_update_dpp((int)k, (int)k, 0x111, 0xF, 0xF, false));
  k = max(k, (uint32_t)__builtin_amdgcn_update_dpp((int)k, (int)k, 0x112, 0xF, 0xF, false));
  k = max(k, (uint32_t)__builtin_amdgcn_update_dpp((int)k, (int)k, 0x114, 0xF, 0xF, false));
  k = max(k, (uint32_t)__builtin_amdgcn_update_dpp((int)k, (int)k, 0x118, 0xF, 0xF, false));
  const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)k, 15);
  const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)k, 31);
  const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)k, 47);
  const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)k, 63);
  return max(max(a, b), max(c, d));
}

struct SelectArgs {
  const float* X;
  int ldx;
  int64_t rows;
  int l;
  const int32_t* sel_in;  // nullptr at the leaf level
  const int32_t* cnt_in;
  int64_t nodes_in;
  int32_t* sel_out;
  int32_t* col_out;
  int32_t* cnt_out;
  float* leaf_max;        // per-leaf max |X| (written by the leaf level)
  int64_t nleaves;
  int is_root;
  double tol;
};

template <int LP>
__global__ __launch_bounds__(kNode) void lu_select_kernel(SelectArgs a) {
  __shared__ __align__(16) float piv[2][LP];
  __shared__ float red_v[kWaves];
  __shared__ __align__(16) uint32_t red_k[2][kWaves];
  __shared__ int cand[kNode];
  __shared__ int ncand_s;
  __shared__ float thr_s;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t node = blockIdx.x;
  const bool leaf = a.sel_in == nullptr;
  if (t == 0) {
    int nc = 0;
    if (leaf) {
      nc = (int)min((int64_t)kNode, a.rows - node * kNode);
    } else {
      for (int c = 0; c < kFanIn; ++c) {
        const int64_t ch = kFanIn * node + c;
        if (ch < a.nodes_in) nc += a.cnt_in[ch];
      }
    }
    ncand_s = nc;
  }
  if (leaf) {
    if (t < min((int64_t)kNode, a.rows - node * kNode)) cand[t] = (int)(node * kNode + t);
  } else if (t == 0) {
    int o = 0;
    for (int c = 0; c < kFanIn; ++c) {
      const int64_t ch = kFanIn * node + c;
      if (ch >= a.nodes_in) break;
      const int n = a.cnt_in[ch];
      for (int i = 0; i < n; ++i) cand[o + i] = a.sel_in[ch * kMaxL + i];
      o += n;
    }
  }
  __syncthreads();
  const int ncand = ncand_s;
  bool act = t < ncand;
  const int myrow = act ? cand[t] : 0;
  float row[LP];
  {
    const float* src = a.X + (size_t)myrow * a.ldx;
    const bool vec = ((a.ldx & 3) == 0) && ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0);
    if (act && vec) {
      static_for<0, LP / 4>([&](auto qc) {
        constexpr int c = 4 * decltype(qc)::value;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c < a.l) v = *reinterpret_cast<const float4*>(src + c);
        row[c] = v.x;
        row[c + 1] = c + 1 < a.l ? v.y : 0.f;
        row[c + 2] = c + 2 < a.l ? v.z : 0.f;
        row[c + 3] = c + 3 < a.l ? v.w : 0.f;
      });
    } else {
      static_for<0, LP>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        row[c] = (act && c < a.l) ? src[c] : 0.f;
      });
    }
  }
  // the largest |entry| of the leaf (for the root's rank threshold)
  if (leaf) {
    float mx = 0.f;
    static_for<0, LP>([&](auto cc) { mx = fmaxf(mx, fabsf(row[decltype(cc)::value])); });
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0) red_v[wave] = mx;
    __syncthreads();
    if (t == 0) {
      float m2 = 0.f;
      for (int w = 0; w < kWaves; ++w) m2 = fmaxf(m2, red_v[w]);
      a.leaf_max[node] = m2;
    }
    __syncthreads();
  }
  if (a.is_root) {
    float mx = 0.f;
    for (int64_t i = t; i < a.nleaves; i += kNode) mx = fmaxf(mx, a.leaf_max[i]);
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0) red_v[wave] = mx;
    __syncthreads();
    if (t == 0) {
      float m2 = 0.f;
      for (int w = 0; w < kWaves; ++w) m2 = fmaxf(m2, red_v[w]);
      thr_s = (float)(a.tol * (double)m2);
    }
    __syncthreads();
  } else if (t == 0) {
    thr_s = 0.f;
  }
  __syncthreads();
  const float thr = thr_s;
  // Elimination in blocks of 8 pivot columns: inside a block the pivot column is the
  // compile-time register row[jr]; after the block the row is shifted left by 8, so a
  // runtime loop over blocks keeps every access to `row` static (no scratch memory). The
  // update runs over whole 8-column chunks; columns left of the pivot are finished and
  // never read again, so updating them is harmless.
  constexpr int NC = LP / 8;
  int cnt = 0;
  for (int jb = 0; jb < NC; ++jb) {
#pragma unroll
    for (int jr = 0; jr < 8; ++jr) {
      const int j = 8 * jb + jr;
      if (j < a.l) {
        // argmax key: |value| with its 9 lowest mantissa bits replaced by (511 - thread), so
        // the maximum picks the largest magnitude (to 2^-14 relative) and, among those, the
        // lowest row slot; retired rows give 0
        const uint32_t key =
            act ? ((__float_as_uint(fabsf(row[jr])) & ~0x1FFu) | (uint32_t)(kNode - 1 - t)) : 0u;
        const uint32_t wk = wave_max_key(key);
        if (lane == 0) red_k[j & 1][wave] = wk;
        __syncthreads();
        uint32_t best = red_k[j & 1][0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) best = max(best, red_k[j & 1][w]);
        const int bw = kNode - 1 - (int)(best & 0x1FFu);
        const float bv = __uint_as_float(best & ~0x1FFu);
        if (bv > thr) {
          float* pr = piv[j & 1];
          float4* pr4 = reinterpret_cast<float4*>(pr);
          if (t == bw) {
#pragma unroll
            for (int c = 0; c < LP; c += 4) pr4[c / 4] = make_float4(row[c], row[c + 1], row[c + 2], row[c + 3]);
            act = false;
            a.sel_out[node * kMaxL + cnt] = myrow;
            a.col_out[node * kMaxL + cnt] = j;
          }
          __syncthreads();
          if (act) {
            // the multiplier only steers which rows survive the tournament (the pivot rows are
            // refactored in FP64 afterwards), so the hardware reciprocal is accurate enough
            const float f = row[jr] * __builtin_amdgcn_rcpf(pr[jr]);
#pragma unroll
            for (int cb = 0; cb < NC; ++cb) {
              if (cb < NC - jb) {
                const float4 p0 = pr4[2 * cb], p1 = pr4[2 * cb + 1];  // broadcast 16-byte reads
                const int c = 8 * cb;
                row[c + 0] = fmaf(-f, p0.x, row[c + 0]);
                row[c + 1] = fmaf(-f, p0.y, row[c + 1]);
                row[c + 2] = fmaf(-f, p0.z, row[c + 2]);
                row[c + 3] = fmaf(-f, p0.w, row[c + 3]);
                row[c + 4] = fmaf(-f, p1.x, row[c + 4]);
                row[c + 5] = fmaf(-f, p1.y, row[c + 5]);
                row[c + 6] = fmaf(-f, p1.z, row[c + 6]);
                row[c + 7] = fmaf(-f, p1.w, row[c + 7]);
              }
            }
          }
          ++cnt;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < LP - 8; ++c) row[c] = row[c + 8];
#pragma unroll
    for (int c = LP - 8; c < LP; ++c) row[c] = 0.f;
  }
  if (t == 0) a.cnt_out[node] = cnt;
}

// Factor the root's pivot rows without further pivoting in FP64, invert U in place and
// scatter U^-1 into B (l x ldb). One workgroup of 1024 threads on an r x r block in LDS with an
// odd row stride (kMS doubles):
//  * Doolittle: at step s the multipliers of column s are formed, then the trailing block is
//    updated by 8 row phases x 128 columns (a wave covers 64 consecutive columns of one row).
//  * U^-1 column by column (T[j][j] = 1/U[j][j], T[0:j, j] = -T[j][j] T[0:j, 0:j] U[0:j, j],
//    the already inverted leading block in place): eight lanes per row share each dot product.
constexpr int kMS = kMaxL + 1;
constexpr int kFT = 1024;
__global__ __launch_bounds__(kFT) void lu_factor_kernel(const float* X, int ldx, int l, const int32_t* sel,
                                                        const int32_t* selcol, const int32_t* cnt_p, double* B,
                                                        int ldb, int* ndropped) {
  __shared__ double M[kMaxL * kMS];
  __shared__ int colpos[kMaxL];
  __shared__ int colid[kMaxL];
  __shared__ int selrow[kMaxL];
  const int t = threadIdx.x;
  const int r = *cnt_p;
  if (t < kMaxL) colpos[t] = -1;
  __syncthreads();
  if (t < r) {
    colid[t] = selcol[t];
    colpos[selcol[t]] = t;
    selrow[t] = sel[t];
  }
  __syncthreads();
  for (int idx = t; idx < r * r; idx += kFT) {
    const int i = idx / r, j = idx - i * r;
    M[i * kMS + j] = (double)X[(size_t)selrow[i] * ldx + colid[j]];
  }
  __syncthreads();
  const int c = t & (kMaxL - 1), g = t >> 7;  // column, row phase 0..7
  for (int s = 0; s + 1 < r; ++s) {
    if (t > s && t < r) M[t * kMS + s] /= M[s * kMS + s];
    __syncthreads();
    if (c > s && c < r) {
      const double us = M[s * kMS + c];
      for (int i = s + 1 + g; i < r; i += 8) M[i * kMS + c] -= M[i * kMS + s] * us;
    }
    __syncthreads();
  }
  {
    const int i = t >> 3, part = t & 7;
    for (int j = 0; j < r; ++j) {
      double y = 0.0;
      if (i < j) {
        const double* Ti = M + i * kMS;
        for (int k = i + part; k < j; k += 8) y += Ti[k] * M[k * kMS + j];
      }
      y += __shfl_xor(y, 1);
      y += __shfl_xor(y, 2);
      y += __shfl_xor(y, 4);
      const double djj = 1.0 / M[j * kMS + j];
      __syncthreads();  // every read of column j precedes the writes below
      if (i < j && part == 0) M[i * kMS + j] = -djj * y;
      if (t == 0) M[j * kMS + j] = djj;
      __syncthreads();
    }
  }
  for (int idx = t; idx < l * ldb; idx += kFT) {
    const int a = idx / ldb, b = idx - a * ldb;
    double v = 0.0;
    if (b < l) {
      const int pa = colpos[a], pb = colpos[b];
      if (pa >= 0 && pb >= 0 && pa <= pb) v = M[pa * kMS + pb];
    }
    B[idx] = v;
  }
  if (t == 0 && ndropped) *ndropped = l - r;
}

template <int LP>
void select_launch(unsigned nodes, const SelectArgs& a, hipStream_t st) {
  lu_select_kernel<LP><<<nodes, kNode, 0, st>>>(a);
}

}  // namespace

size_t lu_temp_bytes(int64_t rows, int l) {
  (void)l;
  const int64_t leaves = (rows + kNode - 1) / kNode;
  const size_t per = (size_t)leaves * kMaxL * 2 * sizeof(int32_t) + (size_t)leaves * sizeof(int32_t) + 1024;
  return 2 * per + (size_t)leaves * sizeof(float) + 1024;
}

void launch_lu_coeffs(const float* X, int ldx, int64_t rows, int l, double tol, double* B, int ldb, void* temp,
                      int* ndropped_dev, hipStream_t st) {
  const int64_t leaves = (rows + kNode - 1) / kNode;
  char* p = static_cast<char*>(temp);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) / 256 * 256;
    return q;
  };
  int32_t* sel[2];
  int32_t* col[2];
  int32_t* cnt[2];
  for (int b = 0; b < 2; ++b) {
    sel[b] = reinterpret_cast<int32_t*>(take((size_t)leaves * kMaxL * sizeof(int32_t)));
    col[b] = reinterpret_cast<int32_t*>(take((size_t)leaves * kMaxL * sizeof(int32_t)));
    cnt[b] = reinterpret_cast<int32_t*>(take((size_t)leaves * sizeof(int32_t)));
  }
  float* leaf_max = reinterpret_cast<float*>(take((size_t)leaves * sizeof(float)));
  const int lp = panel_ld(l);
  int64_t nodes = leaves;
  int cur = 0;
  SelectArgs a{X, ldx, rows, l, nullptr, nullptr, 0, sel[0], col[0], cnt[0], leaf_max, leaves,
               nodes == 1 ? 1 : 0, tol};
  auto run = [&](unsigned n) {
    switch (lp) {
      case 32: select_launch<32>(n, a, st); break;
      case 64: select_launch<64>(n, a, st); break;
      case 96: select_launch<96>(n, a, st); break;
      default: select_launch<128>(n, a, st); break;
    }
  };
  run((unsigned)nodes);
  while (nodes > 1) {
    const int64_t next = (nodes + kFanIn - 1) / kFanIn;
    a.sel_in = sel[cur];
    a.cnt_in = cnt[cur];
    a.nodes_in = nodes;
    a.sel_out = sel[1 - cur];
    a.col_out = col[1 - cur];
    a.cnt_out = cnt[1 - cur];
    a.is_root = next == 1 ? 1 : 0;
    run((unsigned)next);
    cur = 1 - cur;
    nodes = next;
  }
  lu_factor_kernel<<<1, kFT, 0, st>>>(X, ldx, l, sel[cur], col[cur], cnt[cur], B, ldb, ndropped_dev);
}

}  // namespace frpca
