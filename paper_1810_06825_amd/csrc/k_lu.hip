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

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
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
  __shared__ int red_w[kWaves];
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
        float v = act ? fabsf(row[jr]) : -1.0f;
        int who = t;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const float ov = __shfl_xor(v, off);
          const int ow = __shfl_xor(who, off);
          if (ov > v || (ov == v && ow < who)) {
            v = ov;
            who = ow;
          }
        }
        if (lane == 0) {
          red_v[wave] = v;
          red_w[wave] = who;
        }
        __syncthreads();
        float bv = red_v[0];
        int bw = red_w[0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
          const float ov = red_v[w];
          const int ow = red_w[w];
          if (ov > bv || (ov == bv && ow < bw)) {
            bv = ov;
            bw = ow;
          }
        }
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
            const float f = row[jr] / pr[jr];
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
// scatter U^-1 into B (l x ldb). Thread u owns row u of the r x r pivot block; the LDS row
// stride is odd (kMS doubles) so a column access by all threads hits distinct banks.
constexpr int kMS = kMaxL + 1;
__global__ __launch_bounds__(256) void lu_factor_kernel(const float* X, int ldx, int l, const int32_t* sel,
                                                        const int32_t* selcol, const int32_t* cnt_p, double* B,
                                                        int ldb, int* ndropped) {
  __shared__ double M[kMaxL * kMS];
  __shared__ int colpos[kMaxL];
  __shared__ int colid[kMaxL];
  const int t = threadIdx.x;
  const int r = *cnt_p;
  if (t < kMaxL) colpos[t] = -1;
  __syncthreads();
  if (t < r) {
    colid[t] = selcol[t];
    colpos[selcol[t]] = t;
  }
  __syncthreads();
  if (t < r) {
    const float* src = X + (size_t)sel[t] * ldx;
    for (int j = 0; j < r; ++j) M[t * kMS + j] = (double)src[colid[j]];
  }
  __syncthreads();
  // Doolittle elimination: after step s, row s holds row s of U
  for (int s = 0; s < r; ++s) {
    if (t > s && t < r) {
      const double f = M[t * kMS + s] / M[s * kMS + s];
      for (int v = s + 1; v < r; ++v) M[t * kMS + v] -= f * M[s * kMS + v];
    }
    __syncthreads();
  }
  // in-place inverse of the upper triangle, bottom row first: thread j computes T[i][j]
  for (int i = r - 1; i >= 0; --i) {
    double val = 0.0;
    const int j = t;
    if (j >= i && j < r) {
      const double dinv = 1.0 / M[i * kMS + i];
      if (j == i) {
        val = dinv;
      } else {
        double acc = 0.0;
        for (int k = i + 1; k <= j; ++k) acc += M[i * kMS + k] * M[k * kMS + j];
        val = -dinv * acc;
      }
    }
    __syncthreads();
    if (j >= i && j < r) M[i * kMS + j] = val;
    __syncthreads();
  }
  for (int a = 0; a < l; ++a) {
    for (int b = t; b < ldb; b += 256) {
      double v = 0.0;
      if (b < l) {
        const int pa = colpos[a], pb = colpos[b];
        if (pa >= 0 && pb >= 0 && pa <= pb) v = M[pa * kMS + pb];
      }
      B[(size_t)a * ldb + b] = v;
    }
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
  lu_factor_kernel<<<1, 256, 0, st>>>(X, ldx, l, sel[cur], col[cur], cnt[cur], B, ldb, ndropped_dev);
}

}  // namespace frpca
