// LU basis of Lemma 3 / eq. (8): Q = P^T L for P X = L U, i.e. Q = X U^-1.
//
// Pivot rows are chosen by tournament pivoting (Grigori, Demmel & Xiang, "CALU", SIMAX
// 2011): leaves of 512 rows each run Gaussian elimination with partial pivoting (GEPP), one
// row per thread held in registers, and keep the <= l rows they pivot on; groups of four
// candidate sets (4 l <= 512 rows) are merged by GEPP again until one set remains. The
// root's GEPP fixes the pivot order and which columns have a usable pivot (best remaining
// |entry| > tol * max|X|; inner nodes only skip exactly-zero columns). A final kernel factors
// the pivot rows (no further pivoting needed) in FP64, inverts U and scatters U^-1
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

// Ends each branch of a selection over register-array elements by a uniform index: without
// it the compiler merges the branches into one dynamically indexed access, which moves the
// whole array to scratch memory.
#define FRPCA_KEEP_BRANCH() asm volatile("")

__device__ __forceinline__ double readlane_d(double v, int l) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// 1/v from the hardware reciprocal refined by two Newton steps (within a few ulps of the IEEE
// quotient): it sits on the serial chain of every elimination step, where the IEEE division
// sequence is several times longer. The multipliers only shape the coefficient matrix, whose
// range is what the basis needs.
__device__ __forceinline__ double recip_nr(double v) {
  double r = __builtin_amdgcn_rcp(v);
  r = fma(fma(-v, r, 1.0), r, r);
  r = fma(fma(-v, r, 1.0), r, r);
  return r;
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
  __shared__ int sel_s[kMaxL], col_s[kMaxL];  // chosen rows and their columns, written out at the end
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
  // chunks per update group: four at the widest panel, whose registers already limit a CU to
  // one block; narrower panels keep one chunk per group, so two blocks still fit on a CU
  constexpr int NG = LP >= 128 ? 4 : 1;
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
            sel_s[cnt] = myrow;
            col_s[cnt] = j;
          }
          __syncthreads();
          if (act) {
            // the multiplier only steers which rows survive the tournament (the pivot rows are
            // refactored in FP64 afterwards), so the hardware reciprocal is accurate enough
            const float f = row[jr] * __builtin_amdgcn_rcpf(pr[jr]);
            // live chunks in groups of NG: a group's broadcast reads issue together (one test
            // per chunk makes each chunk wait for its own reads in turn)
#pragma unroll
            for (int g = 0; g < NC; g += NG) {
              if (g < NC - jb) {
                float4 pv[2 * NG];
#pragma unroll
                for (int u = 0; u < 2 * NG; ++u)
                  if (2 * g + u < 2 * NC) pv[u] = pr4[2 * g + u];
#pragma unroll
                for (int u = 0; u < 2 * NG; ++u) {
                  if (2 * g + u < 2 * NC) {
                    const int c = 4 * (2 * g + u);
                    row[c + 0] = fmaf(-f, pv[u].x, row[c + 0]);
                    row[c + 1] = fmaf(-f, pv[u].y, row[c + 1]);
                    row[c + 2] = fmaf(-f, pv[u].z, row[c + 2]);
                    row[c + 3] = fmaf(-f, pv[u].w, row[c + 3]);
                  }
                }
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
  __syncthreads();
  if (t < cnt) {
    a.sel_out[node * kMaxL + t] = sel_s[t];
    a.col_out[node * kMaxL + t] = col_s[t];
  }
  if (t == 0) a.cnt_out[node] = cnt;
}

// Factor the root's pivot rows without further pivoting in FP64, invert U and scatter U^-1
// into B (l x ldb). One workgroup of 1024 threads: wave w holds columns 8 w .. 8 w + 7 and lane
// L rows 2 L, 2 L + 1 of the r x r block, in registers.
//  * Doolittle: the wave owning column s forms the multipliers of step s and leaves them in
//    LDS; after one barrier every wave with live columns takes row s from lane s / 2 with
//    readlane and updates. The owner of column s + 1 updates it first and publishes step s + 1
//    before the rest of its update. The multipliers are not kept (only U is needed).
//  * U goes to LDS; U^-1 by Gauss-Jordan on [U | I] from the last column back: row s of the
//    right block is scaled by 1/U[s][s] and removed from the rows above with the factors
//    U[i][s]. Each wave owns its columns of the right block and reads only U, so this phase
//    needs no barrier; a wave starts at the first step that touches its columns.
constexpr int kMS = kMaxL + 1;
constexpr int kFT = 1024;
constexpr int kFC = 8;  // columns per wave

__global__ __launch_bounds__(kFT) void lu_factor_kernel(const float* X, int ldx, int l, const int32_t* sel,
                                                        const int32_t* selcol, const int32_t* cnt_p, double* B,
                                                        int ldb, int* ndropped) {
  __shared__ double M[kMaxL * kMS];
  __shared__ __align__(16) double mcol[2][kMaxL];
  __shared__ int colpos[kMaxL];
  __shared__ int colid[kMaxL];
  __shared__ int selrow[kMaxL];
  __shared__ double dinv[kMaxL];  // 1 / U[s][s], formed once for the inversion
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r = *cnt_p;
  if (t < kMaxL) colpos[t] = -1;
  __syncthreads();
  if (t < r) {
    colid[t] = selcol[t];
    colpos[selcol[t]] = t;
    selrow[t] = sel[t];
  }
  __syncthreads();
  const int cb = kFC * w;
  double u[2][kFC];
  static_for<0, 2>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const int row = 2 * lane + i;
    static_for<0, kFC>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      u[i][c] = (row < r && cb + c < r) ? (double)X[(size_t)selrow[row] * ldx + colid[cb + c]] : 0.0;
    });
  });
  // multipliers of step s from column s's values colv (this lane's two rows) by its owner
  auto publish = [&](int s, const double (&colv)[2]) {
    const double mine = (s & 1) ? colv[1] : colv[0];
    const double rp = recip_nr(readlane_d(mine, s >> 1));
    double2 m;
    m.x = 2 * lane > s ? colv[0] * rp : 0.0;
    m.y = 2 * lane + 1 > s ? colv[1] * rp : 0.0;
    reinterpret_cast<double2*>(mcol[s & 1])[lane] = m;
  };
  if (w == 0 && r > 1) {
    const double colv[2] = {u[0][0], u[1][0]};
    publish(0, colv);
  }
#pragma unroll 1
  for (int s = 0; s + 1 < r; ++s) {
    __syncthreads();
    if (w < s / kFC) continue;
    const double2 m = reinterpret_cast<const double2*>(mcol[s & 1])[lane];
    double prow[kFC];
    const int pl = s >> 1;
    if (s & 1) {
      static_for<0, kFC>([&](auto cc) { prow[decltype(cc)::value] = readlane_d(u[1][decltype(cc)::value], pl); });
      FRPCA_KEEP_BRANCH();
    } else {
      static_for<0, kFC>([&](auto cc) { prow[decltype(cc)::value] = readlane_d(u[0][decltype(cc)::value], pl); });
      FRPCA_KEEP_BRANCH();
    }
    auto upd = [&](auto cc) {
      constexpr int c = decltype(cc)::value;
      u[0][c] = fma(-m.x, prow[c], u[0][c]);
      u[1][c] = fma(-m.y, prow[c], u[1][c]);
    };
    const int sn = s + 1, nc = sn % kFC;
    const bool own_next = sn + 1 < r && w == sn / kFC;
    if (own_next) {
      double colv[2];
      static_for<0, kFC>([&](auto cc) {
        if (nc == decltype(cc)::value) {
          upd(cc);
          colv[0] = u[0][decltype(cc)::value];
          colv[1] = u[1][decltype(cc)::value];
          FRPCA_KEEP_BRANCH();
        }
      });
      publish(sn, colv);
    }
    const int skip = own_next ? nc : -1;
    static_for<0, kFC>([&](auto cc) {
      if (decltype(cc)::value != skip) upd(cc);
    });
  }
  // U (upper triangle) to LDS
  static_for<0, 2>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const int row = 2 * lane + i;
    static_for<0, kFC>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if (row < r && cb + c < r) M[row * kMS + cb + c] = u[i][c];
    });
  });
  __syncthreads();
  if (t < r) dinv[t] = 1.0 / M[t * kMS + t];
  __syncthreads();
  double tt[2][kFC];
  static_for<0, 2>([&](auto ic) {
    static_for<0, kFC>([&](auto cc) {
      tt[decltype(ic)::value][decltype(cc)::value] =
          (2 * lane + decltype(ic)::value == cb + decltype(cc)::value) ? 1.0 : 0.0;
    });
  });
  // columns cb .. cb + 7 of U^-1 are zero above... below row cb + 7: steps s > cb + 7 leave them alone
#pragma unroll 1
  for (int s = min(r - 1, cb + kFC - 1); s >= 0; --s) {
    const double rinv = dinv[s];
    const double f0 = 2 * lane < s ? M[(2 * lane) * kMS + s] : 0.0;
    const double f1 = 2 * lane + 1 < s ? M[(2 * lane + 1) * kMS + s] : 0.0;
    const int pl = s >> 1;
    double prow[kFC];
    if (s & 1) {
      static_for<0, kFC>([&](auto cc) { prow[decltype(cc)::value] = readlane_d(tt[1][decltype(cc)::value], pl) * rinv; });
      FRPCA_KEEP_BRANCH();
    } else {
      static_for<0, kFC>([&](auto cc) { prow[decltype(cc)::value] = readlane_d(tt[0][decltype(cc)::value], pl) * rinv; });
      FRPCA_KEEP_BRANCH();
    }
    const bool mine0 = 2 * lane == s, mine1 = 2 * lane + 1 == s;
    static_for<0, kFC>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      tt[0][c] = mine0 ? prow[c] : fma(-f0, prow[c], tt[0][c]);
      tt[1][c] = mine1 ? prow[c] : fma(-f1, prow[c], tt[1][c]);
    });
  }
  __syncthreads();  // every wave is done reading U
  static_for<0, 2>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const int row = 2 * lane + i;
    static_for<0, kFC>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if (row < r && cb + c < r) M[row * kMS + cb + c] = tt[i][c];
    });
  });
  __syncthreads();
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
