// LU basis of Lemma 3 / eq. (8): Q = P^T L for P X = L U, i.e. Q = X U^-1.
//
// Pivot rows are chosen by tournament pivoting (Grigori, Demmel & Xiang, "CALU", SIMAX
// 2011): leaves of 256 rows each run Gaussian elimination with partial pivoting (GEPP) in
// registers, one row per thread, and keep the <= l rows they pivot on; pairs of candidate
// sets are merged by GEPP again until one set remains. The root's GEPP fixes the pivot
// order and which columns have a usable pivot (best remaining |entry| > tol * max|X|;
// inner nodes only skip exactly-zero columns). A final kernel factors the pivot rows
// (no further pivoting needed) in FP64, inverts U in place and scatters U^-1 into an l x l
// coefficient matrix B (zero rows/columns for columns without a pivot), so Q = X B runs on
// the MFMA panel kernel. Any pivot choice gives a P^T L spanning range(X) (Lemma 3); the
// pivot rows of Q form a unit lower-triangular block.
#include "kernels.h"

namespace frpca {
namespace {

constexpr int kLeafRows = 256;
constexpr int kAbsBlocks = 1024;

__global__ __launch_bounds__(256) void absmax_kernel(const float* X, int ldx, int64_t rows, int l, float* part) {
  __shared__ float red[256];
  float m = 0.0f;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)gridDim.x * 256)
    for (int c = 0; c < l; ++c) m = fmaxf(m, fabsf(X[r * ldx + c]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
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
  int is_root;
  double tol;
  const float* absmax_part;
  int absmax_n;
};

template <int LP>
__global__ __launch_bounds__(256) void lu_select_kernel(SelectArgs a) {
  __shared__ float piv[2][LP];
  __shared__ float red_v[4];
  __shared__ int red_w[4];
  __shared__ int cand[256];
  __shared__ int ncand_s;
  __shared__ float thr_s;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t node = blockIdx.x;
  if (t == 0) {
    int nc = 0;
    if (a.sel_in == nullptr) {
      const int64_t r0 = node * kLeafRows;
      nc = (int)min((int64_t)kLeafRows, a.rows - r0);
    } else {
      const int64_t n0 = 2 * node, n1 = 2 * node + 1;
      nc = a.cnt_in[n0] + (n1 < a.nodes_in ? a.cnt_in[n1] : 0);
    }
    ncand_s = nc;
    float thr = 0.0f;
    if (a.is_root) {
      float mx = 0.0f;
      for (int i = 0; i < a.absmax_n; ++i) mx = fmaxf(mx, a.absmax_part[i]);
      thr = (float)(a.tol * (double)mx);
    }
    thr_s = thr;
  }
  __syncthreads();
  const int ncand = ncand_s;
  const float thr = thr_s;
  if (a.sel_in == nullptr) {
    if (t < ncand) cand[t] = (int)(node * kLeafRows + t);
  } else {
    const int64_t n0 = 2 * node;
    const int c0 = a.cnt_in[n0];
    if (t < c0) cand[t] = a.sel_in[n0 * kMaxL + t];
    else if (t < ncand) cand[t] = a.sel_in[(n0 + 1) * kMaxL + (t - c0)];
  }
  __syncthreads();
  bool act = t < ncand;
  const int myrow = act ? cand[t] : 0;
  float row[LP];
#pragma unroll
  for (int c = 0; c < LP; ++c) row[c] = (act && c < a.l) ? a.X[(size_t)myrow * a.ldx + c] : 0.0f;
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < LP; ++j) {
    if (j < a.l) {
      float v = act ? fabsf(row[j]) : -1.0f;
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
      for (int w = 1; w < 4; ++w) {
        const float ov = red_v[w];
        const int ow = red_w[w];
        if (ov > bv || (ov == bv && ow < bw)) {
          bv = ov;
          bw = ow;
        }
      }
      if (bv > thr) {
        if (t == bw) {
#pragma unroll
          for (int c = j; c < LP; ++c) piv[j & 1][c] = row[c];
          act = false;
          a.sel_out[node * kMaxL + cnt] = myrow;
          a.col_out[node * kMaxL + cnt] = j;
        }
        __syncthreads();
        if (act) {
          const float f = row[j] / piv[j & 1][j];
#pragma unroll
          for (int c = j + 1; c < LP; ++c) row[c] = fmaf(-f, piv[j & 1][c], row[c]);
        }
        ++cnt;
      }
    }
  }
  if (t == 0) a.cnt_out[node] = cnt;
}

// Factor the root's pivot rows without further pivoting in FP64, invert U in place and
// scatter U^-1 into B (l x ldb).
__global__ __launch_bounds__(256) void lu_factor_kernel(const float* X, int ldx, int l, const int32_t* sel,
                                                        const int32_t* selcol, const int32_t* cnt_p, double* B,
                                                        int ldb, int* ndropped) {
  __shared__ double M[kMaxL * kMaxL];
  __shared__ int colpos[kMaxL];
  __shared__ int rowid[kMaxL], colid[kMaxL];
  const int t = threadIdx.x;
  const int r = *cnt_p;
  for (int c = t; c < kMaxL; c += 256) colpos[c] = -1;
  __syncthreads();
  for (int i = t; i < r; i += 256) {
    rowid[i] = sel[i];
    colid[i] = selcol[i];
    colpos[selcol[i]] = i;
  }
  __syncthreads();
  for (int idx = t; idx < r * r; idx += 256) {
    const int i = idx / r, j = idx - i * r;
    M[i * kMaxL + j] = (double)X[(size_t)rowid[i] * ldx + colid[j]];
  }
  __syncthreads();
  // Doolittle elimination: after step s, row s holds U's row s
  for (int s = 0; s < r; ++s) {
    const double inv = 1.0 / M[s * kMaxL + s];
    const int n = r - s - 1;
    for (int idx = t; idx < n * n; idx += 256) {
      const int u = s + 1 + idx / n, v = s + 1 + idx % n;
      M[u * kMaxL + v] -= (M[u * kMaxL + s] * inv) * M[s * kMaxL + v];
    }
    __syncthreads();
  }
  // in-place inverse of the upper triangle, bottom row first
  for (int i = r - 1; i >= 0; --i) {
    double val = 0.0;
    const int j = i + t;
    const double dinv = 1.0 / M[i * kMaxL + i];
    if (j < r) {
      if (j == i) {
        val = dinv;
      } else {
        double acc = 0.0;
        for (int k = i + 1; k <= j; ++k) acc += M[i * kMaxL + k] * M[k * kMaxL + j];
        val = -dinv * acc;
      }
    }
    __syncthreads();
    if (j < r) M[i * kMaxL + j] = val;
    __syncthreads();
  }
  for (int idx = t; idx < l * ldb; idx += 256) {
    const int a = idx / ldb, b = idx - a * ldb;
    double v = 0.0;
    if (b < l) {
      const int pa = colpos[a], pb = colpos[b];
      if (pa >= 0 && pb >= 0 && pa <= pb) v = M[pa * kMaxL + pb];
    }
    B[idx] = v;
  }
  if (t == 0 && ndropped) *ndropped = l - r;
}

template <int LP>
void select_launch(unsigned nodes, const SelectArgs& a, hipStream_t st) {
  lu_select_kernel<LP><<<nodes, 256, 0, st>>>(a);
}

}  // namespace

size_t lu_temp_bytes(int64_t rows, int l) {
  (void)l;
  const int64_t leaves = (rows + kLeafRows - 1) / kLeafRows;
  const size_t per = (size_t)leaves * kMaxL * 2 * sizeof(int32_t) + (size_t)leaves * sizeof(int32_t) + 256;
  return 2 * per + kAbsBlocks * sizeof(float) + 512;
}

void launch_lu_coeffs(const float* X, int ldx, int64_t rows, int l, double tol, double* B, int ldb, void* temp,
                      int* ndropped_dev, hipStream_t st) {
  const int64_t leaves = (rows + kLeafRows - 1) / kLeafRows;
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
  float* absp = reinterpret_cast<float*>(take(kAbsBlocks * sizeof(float)));
  int absn = (int)min((int64_t)kAbsBlocks, (rows + 255) / 256);
  if (absn < 1) absn = 1;
  absmax_kernel<<<absn, 256, 0, st>>>(X, ldx, rows, l, absp);
  const int lp = panel_ld(l);
  int64_t nodes = leaves;
  int cur = 0;
  SelectArgs a{X, ldx, rows, l, nullptr, nullptr, 0, sel[0], col[0], cnt[0], nodes == 1 ? 1 : 0, tol, absp, absn};
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
    const int64_t next = (nodes + 1) / 2;
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
