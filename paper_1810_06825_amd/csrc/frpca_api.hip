// C interface and host orchestration of frPCA / frPCAt (Alg. 5 / Alg. 6) on gfx950.
//
// Both algorithms are driven by one schedule written for "the short side" (the smaller of
// m, n, where the basis Q lives) and "the long side": the forward product maps a short-side
// panel to the long side (A Q in Alg. 6, A^T Q in Alg. 5) and the back product maps it
// back (A^T Y in Alg. 6, A Y in Alg. 5). Alg. 5 on A is the same computation as Alg. 6 on
// A^T with U and V exchanged, so only the roles of the CSR matrix and its column-major
// mirror swap. Every step is a kernel enqueued on the handle's stream; the host only
// sequences launches.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

using namespace frpca;

namespace {

thread_local std::string g_last_error;
constexpr double kInnerTol = 1e-12;
constexpr double kDefaultRankTol = 1e-5;
// Cholesky pivot guard of orth() in the basic algorithms: a column whose residual norm falls
// below about 3e-7 of its own norm is numerically dependent on the earlier ones.
constexpr double kCholTol = 1e-13;
// degree of the Chebyshev filter between Rayleigh-Ritz steps of eigSVDs
constexpr int kChebDegree = 8;
// residual level below which FP32 panels cannot resolve a Ritz pair, relative to theta_max
constexpr double kResFloor = 2e-7;

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bump allocator over one device allocation.
struct Arena {
  char* base = nullptr;
  size_t used = 0;
  template <class T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += align256(count * sizeof(T));
    return p;
  }
};

struct DeviceTemp {
  void* p = nullptr;
  explicit DeviceTemp(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{FRPCA_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
  }
  ~DeviceTemp() {
    if (p) (void)hipFree(p);
  }
  DeviceTemp(const DeviceTemp&) = delete;
  DeviceTemp& operator=(const DeviceTemp&) = delete;
};

__global__ void iota_kernel(uint32_t* v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (uint32_t)i;
}
__global__ void widen_kernel(const int32_t* a, int64_t n, int64_t* b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

int bits_for(int64_t maxval) {
  int b = 1;
  while (b < 32 && ((int64_t)1 << b) <= maxval) ++b;
  return b;
}

}  // namespace

struct frpca_ctx {
  int64_t m = 0, n = 0, nnz = 0;
  const int64_t* row_ptr = nullptr;
  const int32_t* col = nullptr;
  const float* val = nullptr;
  hipStream_t stream = nullptr;
  frpca_opts opts{};
  double rank_tol = kDefaultRankTol;

  std::vector<void*> owned;  // setup allocations
  int32_t* rp32 = nullptr;
  int32_t* cp32 = nullptr;
  int32_t* row_csc = nullptr;
  int32_t* perm = nullptr;
  float* val_csc = nullptr;
  MergePlan csr, csc;
  // blocked column order for A^T Y with a long gathered panel (k_bcsc.hip); absent when no
  // column is hot
  bool has_bcsc = false;
  MergePlan bhotp, btailp;  // hot segments (sweep mode) and tail columns
  int32_t *bptr = nullptr, *bptr_tail = nullptr, *brow = nullptr, *bsrc = nullptr, *colmap = nullptr;
  int32_t *bhotcol = nullptr, *btailcol = nullptr;  // hot / tail index -> column
  // centred products (opts.center): column means of A, and the rank-1 term's vector with its
  // reduction partials (k_center.hip)
  float* mu = nullptr;
  float* cvec = nullptr;
  double* cpart = nullptr;
  float* bval = nullptr;
  int64_t bhot = 0, bnblk = 0, bnseg = 0;

  // forward-run workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int ws_lp = 0;
  int ws_bf16 = -1;
  float *Q = nullptr, *X = nullptr, *Y = nullptr, *Z = nullptr;
  uint16_t *Qb = nullptr, *Yb = nullptr;
  double *gram_part = nullptr, *G = nullptr, *W = nullptr, *d = nullptr;
  double *B1 = nullptr, *B2 = nullptr;
  double *R1 = nullptr, *R2 = nullptr, *Rp = nullptr;  // CholeskyQR2 factors (basic algorithms)
  // second long-side panel of the basic algorithms (their bases may live on the long side)
  void* ws2 = nullptr;
  size_t ws2_bytes = 0;
  int ws2_lp = 0;
  float* Z2 = nullptr;
  // two more short-side panels, the residual partials and the residuals of eigSVDs
  void* ws3 = nullptr;
  size_t ws3_bytes = 0;
  int ws3_lp = 0;
  float *S3 = nullptr, *S4 = nullptr;
  double *res_tmp = nullptr, *res = nullptr;
  float* Skeep = nullptr;  // singular values of the last run (library copy)
  int *order = nullptr, *ndrop = nullptr;
  double* eig_tmp = nullptr;
  float* bpart = nullptr;  // partial rows of the blocked transpose product
  void *lu_tmp = nullptr, *sign_tmp = nullptr;

  // Factors of the last frpca_run, kept for frpca_backward: the long-side panel Z, the
  // short-side basis Q, the final coefficients B1 (long) and B2 (short) with the sign
  // convention folded in, and S. U and V are rebuilt from them (U = Z B1, V = Q B2 for
  // Alg. 6; swapped for Alg. 5). saved_k = 0: no valid factors.
  int saved_k = 0, saved_l = 0, saved_ld = 0;  // k, l and panel leading dimension of that run

  // backward workspace
  void* bws = nullptr;
  size_t bws_bytes = 0;
  int bws_k = 0;

  // ordering of work when the caller switches streams
  hipEvent_t handoff = nullptr;

  frpca_info info{};
  struct Pending {
    hipEvent_t a, b;
    int cls;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::string last_error;

  size_t setup_bytes = 0;

  ~frpca_ctx() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
    if (handoff) (void)hipEventDestroy(handoff);
    for (void* p : owned) (void)hipFree(p);
    if (ws) (void)hipFree(ws);
    if (bws) (void)hipFree(bws);
    if (ws2) (void)hipFree(ws2);
    if (ws3) (void)hipFree(ws3);
  }

  void* alloc_owned(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{FRPCA_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    owned.push_back(p);
    setup_bytes += bytes;
    return p;
  }

  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    FRPCA_HIP(hipEventCreate(&e));
    return e;
  }

  // RAII timing of one kernel class on the handle's stream (when opts.timing is set).
  struct Scope {
    frpca_ctx* h;
    int cls;
    hipEvent_t a = nullptr;
    Scope(frpca_ctx* h_, int cls_) : h(h_), cls(cls_) {
      if (h->opts.timing) {
        a = h->get_event();
        FRPCA_HIP(hipEventRecord(a, h->stream));
      }
    }
    ~Scope() {
      if (a) {
        hipEvent_t b = h->get_event();
        (void)hipEventRecord(b, h->stream);
        h->pending.push_back({a, b, cls});
      }
    }
  };

  void collect_timers() {
    if (pending.empty()) return;
    FRPCA_HIP(hipStreamSynchronize(stream));
    for (auto& p : pending) {
      float ms = 0.f;
      FRPCA_HIP(hipEventElapsedTime(&ms, p.a, p.b));
      info.t_ms[p.cls] += ms;
      info.t_count[p.cls] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }

  void build_plan(MergePlan& p, const int32_t* ptr, const int32_t* idx, const float* v, int64_t nseg,
                  bool sweep = false, int64_t plan_nnz = -1, int64_t sweep_ipw = kSweepItemsPerWave) {
    p.ptr = ptr;
    p.idx = idx;
    p.val = v;
    p.nseg = nseg;
    p.nnz = plan_nnz >= 0 ? plan_nnz : nnz;
    p.sweep = sweep ? 1 : 0;
    p.ipw = sweep ? sweep_ipw : merge_items_per_wave(nseg, p.nnz);
    p.nwaves = std::max<int64_t>(1, (nseg + p.nnz + p.ipw - 1) / p.ipw);
    p.part_seg = static_cast<int32_t*>(alloc_owned((p.nwaves + 1) * sizeof(int32_t)));
    p.part_e = static_cast<int32_t*>(alloc_owned((p.nwaves + 1) * sizeof(int32_t)));
    p.fix_w0 = static_cast<int32_t*>(alloc_owned(p.nwaves * sizeof(int32_t)));
    p.carry = static_cast<float*>(alloc_owned(p.nwaves * 128 * sizeof(float)));
    p.head = static_cast<float*>(alloc_owned(p.nwaves * 128 * sizeof(float)));
    if (sweep) p.sweep_ctr = static_cast<int32_t*>(alloc_owned(8 * 32 * sizeof(int32_t)));
    launch_merge_partition(p, stream);
    launch_merge_fixplan(p, stream);
  }

  // A^T in through the blocked order: the hot segments into the partial rows, the tail columns
  // straight into their rows of out (n x ld_out), then the fixed-order combine of the hot rows
  void bcsc_product(int lp, const void* in, bool in_bf16, int ld_in, float* part, float* out32, uint16_t* out16,
                    int ld_out, hipStream_t st) {
    launch_spmm(bhotp, lp, in, in_bf16, ld_in, part, nullptr, lp, st);
    launch_spmm(btailp, lp, in, in_bf16, ld_in, out32, out16, ld_out, st);
    launch_bcsc_combine(part, lp, bhotcol, bhot, bnblk, lp, out32, out16, ld_out, st);
  }

  int64_t short_rows() const { return std::min(m, n); }
  int64_t long_rows() const { return std::max(m, n); }

  void ensure_workspace(int lp, int bf16) {
    if (ws && ws_lp >= lp && ws_bf16 == bf16) return;
    if (ws) {
      FRPCA_HIP(hipStreamSynchronize(stream));
      FRPCA_HIP(hipFree(ws));
      ws = nullptr;
      ws_bytes = 0;
      saved_k = 0;
    }
    const int64_t Ns = short_rows(), Nl = long_rows();
    auto plan = [&](Arena& a) {
      Q = a.take<float>((size_t)Ns * lp);
      X = a.take<float>((size_t)Ns * lp);
      Qb = bf16 ? a.take<uint16_t>((size_t)Ns * lp) : nullptr;
      Z = a.take<float>((size_t)Nl * lp);
      Y = Z;  // FP32 long-side panel of the inner passes (those not stored in BF16)
      Yb = bf16 ? a.take<uint16_t>((size_t)Nl * lp) : nullptr;
      gram_part = a.take<double>(gram_partial_bytes(lp) / sizeof(double));
      G = a.take<double>(kMaxL * kMaxL);
      W = a.take<double>(kMaxL * kMaxL);
      B1 = a.take<double>(kMaxL * kMaxL);
      B2 = a.take<double>(kMaxL * kMaxL);
      R1 = a.take<double>(kMaxL * kMaxL);
      R2 = a.take<double>(kMaxL * kMaxL);
      Rp = a.take<double>(kMaxL * kMaxL);
      Skeep = a.take<float>(kMaxL);
      d = a.take<double>(kMaxL);
      order = a.take<int>(kMaxL);
      eig_tmp = a.take<double>(eig_scratch_bytes() / sizeof(double));
      ndrop = a.take<int>(4);
      lu_tmp = a.take<char>(lu_temp_bytes(Ns, lp));
      sign_tmp = a.take<char>(sign_partial_bytes(Nl, kMaxL));
      bpart = has_bcsc ? a.take<float>((size_t)bhotp.nseg * lp) : nullptr;
      cvec = opts.center ? a.take<float>(kMaxL) : nullptr;
      cpart = opts.center ? a.take<double>(wsum_temp_bytes(std::max(m, n)) / sizeof(double)) : nullptr;
    };
    Arena probe;
    plan(probe);
    const size_t need = probe.used;
    if (opts.max_workspace && need + setup_bytes > opts.max_workspace)
      throw Error{FRPCA_ENOMEM, "workspace of " + std::to_string(need) + " bytes exceeds opts.max_workspace"};
    if (hipMalloc(&ws, need) != hipSuccess) {
      (void)hipGetLastError();
      ws = nullptr;
      throw Error{FRPCA_ENOMEM, "workspace allocation of " + std::to_string(need) + " bytes failed"};
    }
    Arena real;
    real.base = static_cast<char*>(ws);
    plan(real);
    ws_bytes = need;
    ws_lp = lp;
    ws_bf16 = bf16;
  }

  void ensure_long2(int lp) {
    if (ws2 && ws2_lp >= lp) return;
    if (ws2) {
      FRPCA_HIP(hipStreamSynchronize(stream));
      FRPCA_HIP(hipFree(ws2));
      ws2 = nullptr;
      ws2_bytes = 0;
    }
    const size_t need = align256((size_t)long_rows() * lp * sizeof(float));
    if (opts.max_workspace && need + ws_bytes + setup_bytes > opts.max_workspace)
      throw Error{FRPCA_ENOMEM, "second long-side panel of " + std::to_string(need) + " bytes exceeds opts.max_workspace"};
    if (hipMalloc(&ws2, need) != hipSuccess) {
      (void)hipGetLastError();
      ws2 = nullptr;
      throw Error{FRPCA_ENOMEM, "long-side panel allocation of " + std::to_string(need) + " bytes failed"};
    }
    ws2_bytes = need;
    ws2_lp = lp;
    Z2 = static_cast<float*>(ws2);
  }

  void ensure_short2(int lp) {
    if (ws3 && ws3_lp >= lp) return;
    if (ws3) {
      FRPCA_HIP(hipStreamSynchronize(stream));
      FRPCA_HIP(hipFree(ws3));
      ws3 = nullptr;
      ws3_bytes = 0;
    }
    auto plan = [&](Arena& a) {
      S3 = a.take<float>((size_t)short_rows() * lp);
      S4 = a.take<float>((size_t)short_rows() * lp);
      res_tmp = a.take<double>(resid_temp_bytes(short_rows()) / sizeof(double));
      res = a.take<double>(kMaxL);
    };
    Arena probe;
    plan(probe);
    const size_t need = probe.used;
    if (opts.max_workspace && need + ws_bytes + ws2_bytes + setup_bytes > opts.max_workspace)
      throw Error{FRPCA_ENOMEM, "eigSVDs panels of " + std::to_string(need) + " bytes exceed opts.max_workspace"};
    if (hipMalloc(&ws3, need) != hipSuccess) {
      (void)hipGetLastError();
      ws3 = nullptr;
      throw Error{FRPCA_ENOMEM, "eigSVDs panel allocation of " + std::to_string(need) + " bytes failed"};
    }
    Arena real;
    real.base = static_cast<char*>(ws3);
    plan(real);
    ws3_bytes = need;
    ws3_lp = lp;
  }

  // orth() of the basic algorithms on a panel (rows x l, ld lp) in place, through tmp:
  // CholeskyQR2. With Rout, also R = R2 R1 (the triangular factor of the panel).
  void orth_cqr2(float* P, float* tmp, int64_t rows, int l, int lp, double* Rout, hipStream_t st) {
    for (int pass = 0; pass < 2; ++pass) {
      const float* in = pass == 0 ? P : tmp;
      float* out = pass == 0 ? tmp : P;
      double* Bc = pass == 0 ? B1 : B2;
      double* Rc = pass == 0 ? R1 : R2;
      {
        Scope t(this, FRPCA_T_GRAM);
        launch_gram(in, false, lp, nullptr, 0, rows, l, gram_part, G, l, st, false);
      }
      {
        Scope t(this, FRPCA_T_QR);
        launch_chol_inv(G, l, l, kCholTol, Bc, lp, Rout ? Rc : nullptr, nullptr, st);
      }
      if (Rout && pass == 1) {
        Scope t(this, FRPCA_T_QR);
        launch_small_matmul(R2, R1, l, Rout, st);
        return;  // the factor is all the SVD step needs
      }
      Scope t(this, FRPCA_T_TSMM);
      launch_tsmm(in, false, lp, rows, l, Bc, lp, l, lp, out, lp, nullptr, 0, st);
    }
  }
};

namespace {

int fail(frpca_t h, const Error& e) {
  if (h) h->last_error = e.msg;
  else g_last_error = e.msg;
  return e.code;
}

template <class F>
int guarded(frpca_t h, F&& f) {
  try {
    f();
    return FRPCA_OK;
  } catch (const Error& e) {
    return fail(h, e);
  } catch (const std::exception& e) {
    return fail(h, Error{FRPCA_EHIP, e.what()});
  }
}

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{FRPCA_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e)};
}

}  // namespace

extern "C" {

int frpca_create(frpca_t* out, int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                 const float* val, const frpca_opts* opts, void* stream) {
  if (out) *out = nullptr;
  frpca_ctx* h = nullptr;
  int rc = guarded(nullptr, [&] {
    FRPCA_CHECK(out != nullptr, FRPCA_EINVAL, "out handle pointer is NULL");
    FRPCA_CHECK(m >= 1 && n >= 1 && m < INT32_MAX && n < INT32_MAX, FRPCA_EINVAL,
                "need 1 <= m, n < 2^31");
    FRPCA_CHECK(nnz >= 0 && nnz < INT32_MAX, FRPCA_EINVAL, "need 0 <= nnz < 2^31");
    FRPCA_CHECK(row_ptr != nullptr && (nnz == 0 || (col != nullptr && val != nullptr)), FRPCA_EINVAL,
                "NULL CSR array");
    if (opts) FRPCA_CHECK(opts->rank_tol >= 0.0 && opts->rank_tol < 1.0, FRPCA_EINVAL, "rank_tol must be in [0, 1)");
    const auto t0 = std::chrono::steady_clock::now();
    h = new frpca_ctx();
    h->m = m;
    h->n = n;
    h->nnz = nnz;
    h->row_ptr = row_ptr;
    h->col = col;
    h->val = val;
    h->stream = static_cast<hipStream_t>(stream);
    if (opts) h->opts = *opts;
    h->rank_tol = h->opts.rank_tol > 0.0 ? h->opts.rank_tol : kDefaultRankTol;
    hipStream_t st = h->stream;

    {  // validation on the device, one synchronisation
      int* flag = static_cast<int*>(h->alloc_owned(sizeof(int)));
      FRPCA_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
      launch_validate_csr(m, n, nnz, row_ptr, col, val, flag, st);
      check_launch();
      int hflag = 0;
      FRPCA_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
      FRPCA_HIP(hipStreamSynchronize(st));
      if (hflag) {
        std::string why = "malformed CSR:";
        if (hflag & 1) why += " row_ptr[0] != 0 or row_ptr[m] != nnz or out of range;";
        if (hflag & 2) why += " row_ptr decreasing;";
        if (hflag & 4) why += " column index out of [0, n);";
        if (hflag & 8) why += " columns not strictly increasing within a row;";
        if (hflag & 16) why += " non-finite value;";
        throw Error{FRPCA_EINVAL, why};
      }
    }
    h->rp32 = static_cast<int32_t*>(h->alloc_owned((m + 1) * sizeof(int32_t)));
    launch_ptr_to_i32(row_ptr, m + 1, h->rp32, st);
    h->cp32 = static_cast<int32_t*>(h->alloc_owned((n + 1) * sizeof(int32_t)));
    h->row_csc = static_cast<int32_t*>(h->alloc_owned(std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
    h->perm = static_cast<int32_t*>(h->alloc_owned(std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
    h->val_csc = static_cast<float*>(h->alloc_owned(std::max<int64_t>(nnz, 1) * sizeof(float)));
    {
      // stable sort of CSR positions by column gives the column-major order
      const size_t nb = std::max<int64_t>(nnz, 1) * sizeof(uint32_t);
      DeviceTemp keys(nb), keys_alt(nb), vals_alt(nb), row_of(nb);
      DeviceTemp rtmp(radix_temp_bytes(nnz));
      uint32_t* kk = static_cast<uint32_t*>(keys.p);
      uint32_t* vv = reinterpret_cast<uint32_t*>(h->perm);
      if (nnz > 0) {
        FRPCA_HIP(hipMemcpyAsync(kk, col, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        iota_kernel<<<(unsigned)((nnz + 255) / 256), 256, 0, st>>>(vv, nnz);
        radix_sort_pairs(kk, vv, static_cast<uint32_t*>(keys_alt.p), static_cast<uint32_t*>(vals_alt.p), nnz,
                         bits_for(n - 1), rtmp.p, st);
      }
      launch_ptr_from_sorted(kk, nnz, n, h->cp32, st);
      launch_expand_rows(h->rp32, m, nnz, static_cast<int32_t*>(row_of.p), st);
      launch_gather_csc(vv, static_cast<int32_t*>(row_of.p), val, nnz, h->row_csc, h->val_csc, st);
      check_launch();
      h->build_plan(h->csr, h->rp32, col, val, m);
      h->build_plan(h->csc, h->cp32, h->row_csc, h->val_csc, n);
      h->csr.in_rows = n;  // the forward product over rows gathers rows of an n-row panel
      h->csc.in_rows = m;
      if (h->opts.center) {
        h->mu = static_cast<float*>(h->alloc_owned(std::max<int64_t>(n, 1) * sizeof(float)));
        launch_colmean(h->cp32, h->val_csc, n, m, h->mu, st);
      }
      check_launch();
      // blocked column order for the transpose product (hot columns split by row block)
      if (nnz > 0) {
        const int64_t nblk = (m + (1 << kBcscRowShift) - 1) >> kBcscRowShift;
        const int32_t thresh = (int32_t)std::min<int64_t>(INT32_MAX, (int64_t)kHotPerBlock * nblk);
        DeviceTemp hot((n + 1) * sizeof(int32_t)), tail((n + 1) * sizeof(int32_t));
        DeviceTemp hpre((n + 1) * sizeof(int32_t)), tpre((n + 1) * sizeof(int32_t)), stmp(scan_temp_bytes(n));
        launch_hot_flags(h->cp32, n, thresh, static_cast<int32_t*>(hot.p), static_cast<int32_t*>(tail.p), st);
        exclusive_scan_i32(static_cast<int32_t*>(hot.p), static_cast<int32_t*>(hpre.p), n, stmp.p, st);
        exclusive_scan_i32(static_cast<int32_t*>(tail.p), static_cast<int32_t*>(tpre.p), n, stmp.p, st);
        int32_t hh = 0;
        FRPCA_HIP(hipMemcpyAsync(&hh, static_cast<int32_t*>(hpre.p) + n, sizeof(int32_t), hipMemcpyDeviceToHost,
                                 st));
        FRPCA_HIP(hipStreamSynchronize(st));
        const int64_t nhs = nblk * (int64_t)hh, nseg = nhs + (n - hh);
        if (hh > 0 && nseg < INT32_MAX) {
          h->has_bcsc = true;
          h->bhot = hh;
          h->bnblk = nblk;
          h->bnseg = nseg;
          h->colmap = static_cast<int32_t*>(h->alloc_owned(n * sizeof(int32_t)));
          h->bptr = static_cast<int32_t*>(h->alloc_owned((nseg + 1) * sizeof(int32_t)));
          h->brow = static_cast<int32_t*>(h->alloc_owned(nnz * sizeof(int32_t)));
          h->bval = static_cast<float*>(h->alloc_owned(nnz * sizeof(float)));
          launch_colmap(static_cast<int32_t*>(hot.p), static_cast<int32_t*>(hpre.p), static_cast<int32_t*>(tpre.p),
                        n, h->colmap, st);
          h->bhotcol = static_cast<int32_t*>(h->alloc_owned(hh * sizeof(int32_t)));
          h->btailcol = static_cast<int32_t*>(h->alloc_owned(std::max<int64_t>(n - hh, 1) * sizeof(int32_t)));
          launch_colmap_inverse(h->colmap, n, h->bhotcol, h->btailcol, st);
          // the (row block, hot column) runs and the tail columns, read off the mirror
          // (the runs' mirror starts are kept: new values reach the blocked order by the same copies)
          DeviceTemp rcnt((nseg + 1) * sizeof(int32_t)), rscan(scan_temp_bytes(nseg));
          h->bsrc = static_cast<int32_t*>(h->alloc_owned(std::max<int64_t>(nseg, 1) * sizeof(int32_t)));
          int32_t* cnt = static_cast<int32_t*>(rcnt.p);
          launch_bcsc_runs(h->cp32, h->row_csc, h->bhotcol, h->btailcol, hh, nblk, n - hh, kBcscRowShift, cnt,
                           h->bsrc, st);
          exclusive_scan_i32(cnt, h->bptr, nseg, rscan.p, st);
          launch_bcsc_copy(h->bptr, h->bsrc, nseg, h->row_csc, h->val_csc, h->brow, h->bval, st);
          check_launch();
          int32_t nnz_hot = 0;
          FRPCA_HIP(hipMemcpyAsync(&nnz_hot, h->bptr + nhs, sizeof(int32_t), hipMemcpyDeviceToHost, st));
          FRPCA_HIP(hipStreamSynchronize(st));
          h->bptr_tail = static_cast<int32_t*>(h->alloc_owned((n - hh + 1) * sizeof(int32_t)));
          launch_rebase(h->bptr + nhs, n - hh + 1, nnz_hot, h->bptr_tail, st);
          // sweep partitions sized so the band of items in flight (the resident waves, 512 per
          // XCD, each on one partition) covers about two row blocks per XCD, whose rows of Y
          // (2 MB each at l = 128) then stay in that XCD's 4 MB L2
          const int64_t sweep_ipw =
              std::max<int64_t>(kSweepMinIpw, std::min<int64_t>(kSweepItemsPerWave, nnz_hot / nblk / FRPCA_SWEEP_PARTS));
          h->build_plan(h->bhotp, h->bptr, h->brow, h->bval, nhs, true, nnz_hot, sweep_ipw);
          h->build_plan(h->btailp, h->bptr_tail, h->brow + nnz_hot, h->bval + nnz_hot, n - hh, false,
                        nnz - nnz_hot);
          h->btailp.out_row = h->btailcol;  // tail segment i is column btailcol[i] of the result
          h->bhotp.in_rows = h->btailp.in_rows = m;
          check_launch();
        }
      }
      FRPCA_HIP(hipStreamSynchronize(st));
    }
    h->info.m = m;
    h->info.n = n;
    h->info.nnz = nnz;
    h->info.orientation = m >= n ? 6 : 5;
    h->info.hot_cols = h->bhot;
    h->info.row_blocks = h->has_bcsc ? h->bnblk : 0;
    h->info.hot_nnz = h->has_bcsc ? h->bhotp.nnz : 0;
    h->info.create_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
  if (rc != FRPCA_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return FRPCA_OK;
}

int frpca_set_values(frpca_t h, const float* val) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(val != nullptr || h->nnz == 0, FRPCA_EINVAL, "NULL values");
    h->val = val;
    h->csr.val = val;
    h->saved_k = 0;  // the last run's factors belong to the old values
    launch_gather_values(h->perm, val, h->nnz, h->val_csc, h->stream);
    if (h->has_bcsc) launch_bcsc_values(h->bptr, h->bsrc, h->bnseg, h->val_csc, h->bval, h->stream);
    if (h->opts.center) launch_colmean(h->cp32, h->val_csc, h->n, h->m, h->mu, h->stream);
    check_launch();
  });
}

int frpca_set_stream(frpca_t h, void* stream) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    hipStream_t ns = static_cast<hipStream_t>(stream);
    if (ns == h->stream) return;
    // work queued on the old stream uses the handle's buffers: the new stream starts after it
    if (!h->handoff) FRPCA_HIP(hipEventCreateWithFlags(&h->handoff, hipEventDisableTiming));
    FRPCA_HIP(hipEventRecord(h->handoff, h->stream));
    FRPCA_HIP(hipStreamWaitEvent(ns, h->handoff, 0));
    h->stream = ns;
  });
}

int frpca_run(frpca_t h, int k, int p_passes, int s_oversample, uint64_t seed, float* U, float* S, float* V) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    const int64_t m = h->m, n = h->n;
    FRPCA_CHECK(k >= 1 && s_oversample >= 0, FRPCA_EINVAL, "need k >= 1 and s >= 0");
    const int l = k + s_oversample;
    FRPCA_CHECK(l <= std::min(m, n), FRPCA_EINVAL, "need k + s <= min(m, n)");
    FRPCA_CHECK(l <= kMaxL, FRPCA_EINVAL, "need k + s <= 128");
    FRPCA_CHECK(p_passes >= 2, FRPCA_EINVAL, "the pass parameter q must be >= 2 (Alg. 5/6)");
    FRPCA_CHECK(U && S && V, FRPCA_EINVAL, "NULL output");
    const int LP = panel_ld(l);
    const int bfmode = h->opts.panel_bf16;
    FRPCA_CHECK(bfmode >= 0 && bfmode <= 4, FRPCA_EINVAL, "opts.panel_bf16 must be 0 .. 4");
    h->saved_k = 0;
    h->ensure_workspace(LP, bfmode ? 1 : 0);
    // which inner pass pairs store panels in BF16: all of them (modes 1 and 3) or all but the
    // last one, whose basis feeds the final Rayleigh-Ritz step (modes 2 and 4); which panels:
    // the basis read by the forward product and the long-side panel read by the back product
    // (modes 1 and 2), only the basis (mode 3) or only the long-side panel (mode 4)
    const int last = (p_passes - 1) / 2;
    auto bf_pair = [&](int i) { return bfmode == 1 || bfmode == 3 || ((bfmode == 2 || bfmode == 4) && i < last); };
    const bool bf_basis = bfmode != 4;
    const bool bf_long = bfmode != 3;
    const bool fused = h->opts.fused_pass != 0;
    FRPCA_CHECK(!fused || (!h->opts.center && !bfmode), FRPCA_EINVAL,
                "opts.fused_pass does not combine with center or panel_bf16");
    hipStream_t st = h->stream;
    const bool a6 = m >= n;
    const MergePlan& Fp = a6 ? h->csr : h->csc;  // short side -> long side
    const MergePlan& Bp = a6 ? h->csc : h->csr;  // long side -> short side
    const int64_t Ns = h->short_rows(), Nl = h->long_rows();
    const int fwd_cls = FRPCA_T_SPMM_F, back_cls = FRPCA_T_SPMM_B;

    // one product = main merge-path kernel + carry fix-up, timed as separate classes
    auto spmm = [&](const MergePlan& p, int cls, const void* in, bool in_b, float* o32, uint16_t* o16,
                    SpmmCorr corr = {}) {
      {
        frpca_ctx::Scope t(h, cls);
        launch_spmm_main(p, LP, in, in_b, LP, o32, o16, LP, st, corr);
      }
      frpca_ctx::Scope t(h, FRPCA_T_SPMM_FIX);
      launch_spmm_fixup(p, LP, o32, o16, LP, st, corr);
    };
    // centred products (opts.center): the rank-1 term of (A - 1 mu^T) X is 1 (mu^T X) over the
    // n rows of X; that of (A - 1 mu^T)^T Y is mu (1^T Y) over the m rows of Y
    const bool cen = h->opts.center != 0;
    auto corr_a = [&](const void* X, bool xb) -> SpmmCorr {
      if (!cen) return {};
      frpca_ctx::Scope t(h, FRPCA_T_CENTER);
      launch_wsum(X, xb, LP, n, LP, h->mu, 1.0, h->cpart, h->cvec, st);
      return {h->cvec, nullptr};
    };
    auto corr_at = [&](const void* Y, bool yb) -> SpmmCorr {
      if (!cen) return {};
      frpca_ctx::Scope t(h, FRPCA_T_CENTER);
      launch_wsum(Y, yb, LP, m, LP, nullptr, 1.0, h->cpart, h->cvec, st);
      return {h->cvec, h->mu};
    };
    // forward product (short side -> long side): A Q for Alg. 6, A^T Q for Alg. 5
    auto forward_corr = [&](const void* in, bool in_b) { return a6 ? corr_a(in, in_b) : corr_at(in, in_b); };
    auto forward_inner = [&](bool bf) {
      const bool qb = bf && bf_basis, yb = bf && bf_long;
      const void* in = qb ? static_cast<const void*>(h->Qb) : static_cast<const void*>(h->Q);
      spmm(Fp, fwd_cls, in, qb, yb ? nullptr : h->Y, yb ? h->Yb : nullptr, forward_corr(in, qb));
    };
    // back product (long side -> short side). For Alg. 6 the panel Y = (A - 1 mu^T) Q of a
    // centred forward product has 1^T Y = (1^T A - m mu^T) Q = 0 exactly, so the term is
    // skipped there (input_centred); the Gaussian start of even q has it.
    auto back = [&](bool input_centred, bool bf_pass) {
      const bool bf = bf_pass && bf_long;
      const void* in = bf ? static_cast<const void*>(h->Yb) : static_cast<const void*>(h->Y);
      SpmmCorr corr{};
      if (cen && !(a6 && input_centred)) corr = a6 ? corr_at(in, bf != 0) : corr_a(in, bf != 0);
      if (a6 && h->has_bcsc) {
        spmm(h->bhotp, back_cls, in, bf != 0, h->bpart, nullptr);
        spmm(h->btailp, FRPCA_T_SPMM_TAIL, in, bf != 0, h->X, nullptr, corr);
        frpca_ctx::Scope t(h, FRPCA_T_SPMM_COMB);
        launch_bcsc_combine(h->bpart, LP, h->bhotcol, h->bhot, h->bnblk, LP, h->X, nullptr, LP, st, corr);
      } else {
        spmm(Bp, back_cls, in, bf != 0, h->X, nullptr, corr);
      }
    };
    // the new basis also gets a BF16 copy when the next pass pair reads BF16 panels
    auto basis_from_B1 = [&](bool next_bf) {
      frpca_ctx::Scope t(h, FRPCA_T_TSMM);
      launch_tsmm(h->X, false, LP, Ns, l, h->B1, LP, l, LP, h->Q, LP, next_bf ? h->Qb : nullptr, LP, st);
    };
    auto orth_lu = [&](bool next_bf) {
      {
        frpca_ctx::Scope t(h, FRPCA_T_LU);
        launch_lu_coeffs(h->X, LP, Ns, l, kInnerTol, h->B1, LP, h->lu_tmp, h->ndrop + 1, st);
      }
      basis_from_B1(next_bf);
    };
    auto gram_eig = [&](const float* P, int64_t rows) {
      {
        frpca_ctx::Scope t(h, FRPCA_T_GRAM);
        launch_gram(P, false, LP, nullptr, 0, rows, l, h->gram_part, h->G, l, st, h->opts.gram_f32 != 0);
      }
      frpca_ctx::Scope t(h, FRPCA_T_EIG);
      launch_eig(h->G, l, l, h->d, h->W, h->eig_tmp, st);
    };
    auto orth_eig = [&](bool next_bf) {
      gram_eig(h->X, Ns);
      launch_eigsvd_coeffs(h->d, h->W, l, LP, kInnerTol, h->B1, nullptr, st);
      basis_from_B1(next_bf);
    };

    // start of the pass schedule (the start counts as pass pair 0 for the BF16 schedule)
    if (p_passes % 2 == 0) {
      const bool bf0 = bf_pair(0) && bf_long;
      {
        frpca_ctx::Scope t(h, FRPCA_T_GAUSS);  // long-side Gaussian (the transposed randn(k+s, .))
        launch_gaussian(seed, Nl, l, LP, bf0 ? nullptr : h->Y, bf0 ? h->Yb : nullptr, st);
      }
      back(false, bf0);
      if (p_passes == 2) orth_eig(false);
      else orth_lu(bf_pair(1) && bf_basis);
    } else {
      frpca_ctx::Scope t(h, FRPCA_T_GAUSS);
      launch_gaussian(seed, Ns, l, LP, h->Q, last >= 1 && bf_pair(1) && bf_basis ? h->Qb : nullptr, st);
    }
    for (int i = 1; i <= last; ++i) {
      const bool bf = bf_pair(i);
      if (fused) {
        frpca_ctx::Scope t(h, FRPCA_T_SPMM_F);
        launch_fused_pass(Fp.ptr, Fp.idx, Fp.val, Fp.nseg, h->Q, LP, LP, h->X, LP, Ns, st);
      } else {
        forward_inner(bf);
        back(true, bf);
      }
      if (i == last) orth_eig(false);
      else orth_lu(bf_pair(i + 1) && bf_basis);
    }
    // final pass and Rayleigh-Ritz: eigSVD of the long-side panel Z
    spmm(Fp, fwd_cls, h->Q, false, h->Z, nullptr, forward_corr(h->Q, false));
    gram_eig(h->Z, Nl);
    launch_final_coeffs(h->d, h->W, l, k, LP, h->rank_tol, h->B1, h->B2, S, h->Skeep, h->ndrop, st);
    // B1 multiplies the long-side panel Z, B2 the short-side basis Q
    float* out_long = a6 ? U : V;
    float* out_short = a6 ? V : U;
    auto tsmm_long = [&] {
      frpca_ctx::Scope t(h, FRPCA_T_TSMM);
      launch_tsmm(h->Z, false, LP, Nl, l, h->B1, LP, k, k, out_long, k, nullptr, 0, st, nullptr, 0, nullptr, 0,
                  !h->opts.final_f64);
    };
    auto tsmm_short = [&] {
      frpca_ctx::Scope t(h, FRPCA_T_TSMM);
      launch_tsmm(h->Q, false, LP, Ns, l, h->B2, LP, k, k, out_short, k, nullptr, 0, st, nullptr, 0, nullptr, 0,
                  !h->opts.final_f64);
    };
    if (a6) {  // V is the short-side output: build it, fix signs, then U
      tsmm_short();
      if (!h->opts.no_sign_fix) {
        frpca_ctx::Scope t(h, FRPCA_T_SIGN);
        launch_sign_fix(V, n, k, h->B1, h->B2, LP, l, h->sign_tmp, st);
      }
      tsmm_long();
    } else {
      tsmm_long();
      if (!h->opts.no_sign_fix) {
        frpca_ctx::Scope t(h, FRPCA_T_SIGN);
        launch_sign_fix(V, n, k, h->B2, h->B1, LP, l, h->sign_tmp, st);
      }
      tsmm_short();
    }
    check_launch();
    h->info.k = k;
    h->info.s = s_oversample;
    h->info.passes = p_passes;
    h->saved_k = k;
    h->saved_l = l;
    h->saved_ld = LP;
  });
}

int frpca_run_basic(frpca_t h, int k, int p_power, int s_oversample, uint64_t seed, int alg, float* U, float* S,
                    float* V) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    const int64_t m = h->m, n = h->n;
    FRPCA_CHECK(k >= 1 && s_oversample >= 0, FRPCA_EINVAL, "need k >= 1 and s >= 0");
    const int l = k + s_oversample;
    FRPCA_CHECK(l <= std::min(m, n), FRPCA_EINVAL, "need k + s <= min(m, n)");
    FRPCA_CHECK(l <= kMaxL, FRPCA_EINVAL, "need k + s <= 128");
    FRPCA_CHECK(p_power >= 0, FRPCA_EINVAL, "the power parameter p must be >= 0");
    FRPCA_CHECK(alg == 1 || alg == 4, FRPCA_EINVAL, "alg must be 1 (basic rPCA) or 4 (basic rPCAt)");
    FRPCA_CHECK(!h->opts.center, FRPCA_EINVAL, "the centred products apply to frpca_run only");
    FRPCA_CHECK(U && S && V, FRPCA_EINVAL, "NULL output");
    const int LP = panel_ld(l);
    h->saved_k = 0;
    h->ensure_workspace(LP, h->opts.panel_bf16 ? 1 : 0);
    h->ensure_long2(LP);
    hipStream_t st = h->stream;
    const bool a6 = m >= n;
    const MergePlan& Fp = a6 ? h->csr : h->csc;  // short side -> long side
    const MergePlan& Bp = a6 ? h->csc : h->csr;  // long side -> short side
    const int64_t Ns = h->short_rows(), Nl = h->long_rows();
    auto spmm = [&](const MergePlan& p, int cls, const float* in, float* out) {
      {
        frpca_ctx::Scope t(h, cls);
        launch_spmm_main(p, LP, in, false, LP, out, nullptr, LP, st);
      }
      frpca_ctx::Scope t(h, FRPCA_T_SPMM_FIX);
      launch_spmm_fixup(p, LP, out, nullptr, LP, st);
    };
    auto forward = [&](const float* in, float* out) { spmm(Fp, FRPCA_T_SPMM_F, in, out); };
    auto back = [&](const float* in, float* out) {
      if (a6 && h->has_bcsc) {
        spmm(h->bhotp, FRPCA_T_SPMM_B, in, h->bpart);
        spmm(h->btailp, FRPCA_T_SPMM_TAIL, in, out);
        frpca_ctx::Scope t(h, FRPCA_T_SPMM_COMB);
        launch_bcsc_combine(h->bpart, LP, h->bhotcol, h->bhot, h->bnblk, LP, out, nullptr, LP, st);
      } else {
        spmm(Bp, FRPCA_T_SPMM_B, in, out);
      }
    };
    // The basis Q lives on side S (the m side for Alg. 1, the n side for Alg. 4), the Gaussian
    // matrix and G on the other side O. Each side has a panel and a scratch panel for orth().
    const bool s_short = (alg == 4) == a6;
    const int64_t NS = s_short ? Ns : Nl, NO = s_short ? Nl : Ns;
    float* S1 = s_short ? h->Q : h->Z;
    float* S2 = s_short ? h->X : h->Z2;
    float* O1 = s_short ? h->Z : h->Q;
    float* O2 = s_short ? h->Z2 : h->X;
    auto to_S = [&](const float* in, float* out) { s_short ? back(in, out) : forward(in, out); };
    auto to_O = [&](const float* in, float* out) { s_short ? forward(in, out) : back(in, out); };

    {
      frpca_ctx::Scope t(h, FRPCA_T_GAUSS);  // Omega: n x l (Alg. 1), or l x m stored m x l (Alg. 4)
      launch_gaussian(seed, NO, l, LP, O1, nullptr, st);
    }
    to_S(O1, S1);
    h->orth_cqr2(S1, S2, NS, l, LP, nullptr, st);
    for (int i = 0; i < p_power; ++i) {
      to_O(S1, O1);
      h->orth_cqr2(O1, O2, NO, l, LP, nullptr, st);
      to_S(O1, S1);
      h->orth_cqr2(S1, S2, NS, l, LP, nullptr, st);
    }
    // B^T = (the product of Q back to side O); svd(B) from the CholeskyQR2 factor of B^T
    to_O(S1, O1);
    h->orth_cqr2(O1, O2, NO, l, LP, h->Rp, st);
    {
      frpca_ctx::Scope t(h, FRPCA_T_QR);
      launch_jacobi_svd(h->Rp, l, l * 2.220446049250313e-16, h->d, h->W, st);
    }
    // B^T W = (left singular vectors of B^T) diag(sigma): the O-side factor is B^T W / sigma,
    // the S-side factor is Q W (the k largest, largest first)
    double* Bo = h->B1;
    double* Bs = h->B2;
    launch_final_coeffs(h->d, h->W, l, k, LP, h->rank_tol, Bo, Bs, S, h->Skeep, h->ndrop, st);
    const bool u_on_S = alg == 1;  // the m side is S for Alg. 1
    float* Pu = u_on_S ? S1 : O1;
    float* Pv = u_on_S ? O1 : S1;
    double* Bu = u_on_S ? Bs : Bo;
    double* Bv = u_on_S ? Bo : Bs;
    {
      frpca_ctx::Scope t(h, FRPCA_T_TSMM);
      launch_tsmm(Pv, false, LP, n, l, Bv, LP, k, k, V, k, nullptr, 0, st, nullptr, 0, nullptr, 0, !h->opts.final_f64);
    }
    if (!h->opts.no_sign_fix) {
      frpca_ctx::Scope t(h, FRPCA_T_SIGN);
      launch_sign_fix(V, n, k, Bu, Bv, LP, l, h->sign_tmp, st);
    }
    {
      frpca_ctx::Scope t(h, FRPCA_T_TSMM);
      launch_tsmm(Pu, false, LP, m, l, Bu, LP, k, k, U, k, nullptr, 0, st, nullptr, 0, nullptr, 0, !h->opts.final_f64);
    }
    check_launch();
    h->info.k = k;
    h->info.s = s_oversample;
    h->info.passes = 2 * p_power + 2;
  });
}

int frpca_eigsvds(frpca_t h, int k, int s_oversample, uint64_t seed, double tol, int max_iter, float* U, float* S,
                  float* V, int* iters) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    const int64_t m = h->m, n = h->n;
    FRPCA_CHECK(k >= 1 && s_oversample >= 0, FRPCA_EINVAL, "need k >= 1 and s >= 0");
    const int l = k + s_oversample;
    FRPCA_CHECK(l <= std::min(m, n), FRPCA_EINVAL, "need k + s <= min(m, n)");
    FRPCA_CHECK(l <= kMaxL, FRPCA_EINVAL, "need k + s <= 128");
    FRPCA_CHECK(max_iter >= 1, FRPCA_EINVAL, "max_iter must be >= 1");
    FRPCA_CHECK(!h->opts.center, FRPCA_EINVAL, "the centred products apply to frpca_run only");
    FRPCA_CHECK(U && S && V, FRPCA_EINVAL, "NULL output");
    if (tol <= 0.0) tol = 1e-6;
    const int LP = panel_ld(l);
    h->saved_k = 0;
    h->ensure_workspace(LP, h->opts.panel_bf16 ? 1 : 0);
    h->ensure_short2(LP);
    hipStream_t st = h->stream;
    const bool a6 = m >= n;
    const MergePlan& Fp = a6 ? h->csr : h->csc;  // short side -> long side
    const MergePlan& Bp = a6 ? h->csc : h->csr;  // long side -> short side
    const int64_t Ns = h->short_rows(), Nl = h->long_rows();
    auto spmm = [&](const MergePlan& p, int cls, const float* in, float* out) {
      {
        frpca_ctx::Scope t(h, cls);
        launch_spmm_main(p, LP, in, false, LP, out, nullptr, LP, st);
      }
      frpca_ctx::Scope t(h, FRPCA_T_SPMM_FIX);
      launch_spmm_fixup(p, LP, out, nullptr, LP, st);
    };
    auto forward = [&](const float* in, float* out) { spmm(Fp, FRPCA_T_SPMM_F, in, out); };
    auto back = [&](const float* in, float* out) {
      if (a6 && h->has_bcsc) {
        spmm(h->bhotp, FRPCA_T_SPMM_B, in, h->bpart);
        spmm(h->btailp, FRPCA_T_SPMM_TAIL, in, out);
        frpca_ctx::Scope t(h, FRPCA_T_SPMM_COMB);
        launch_bcsc_combine(h->bpart, LP, h->bhotcol, h->bhot, h->bnblk, LP, out, nullptr, LP, st);
      } else {
        spmm(Bp, FRPCA_T_SPMM_B, in, out);
      }
    };
    // B P = A^T (A P) for a short-side panel P (m >= n; A A^T for m < n): B is never formed
    auto apply_B = [&](const float* P, float* out) {
      forward(P, h->Z);
      back(h->Z, out);
    };
    // four short-side panels change roles: the basis, B times it, and two filter iterates
    float* buf[4] = {h->Q, h->X, h->S3, h->S4};
    float* Qc = buf[0];
    {
      frpca_ctx::Scope t(h, FRPCA_T_GAUSS);  // starting block: a Gaussian n x l matrix
      launch_gaussian(seed, Ns, l, LP, Qc, nullptr, st);
    }
    h->orth_cqr2(Qc, buf[1], Ns, l, LP, nullptr, st);
    std::vector<double> r2(l), theta(l), hist;
    int it = 0;
    for (;;) {
      ++it;
      // Rayleigh-Ritz on range(Qc): H = Qc^T B Qc, (theta, W) = eig(H), Ritz vectors Qc W
      float* BQ = Qc == buf[1] ? buf[0] : buf[1];
      apply_B(Qc, BQ);
      {
        frpca_ctx::Scope t(h, FRPCA_T_GRAM);
        launch_gram(Qc, false, LP, BQ, LP, Ns, l, h->gram_part, h->G, l, st, false);
        launch_symmetrize(h->G, l, st);
      }
      {
        frpca_ctx::Scope t(h, FRPCA_T_EIG);
        launch_eig(h->G, l, l, h->d, h->W, h->eig_tmp, st);
      }
      if (it == max_iter) break;
      // residuals of the Ritz pairs: || B (Qc W) - theta (Qc W) || with B (Qc W) = (B Qc) W
      float* R1 = nullptr;
      float* R2 = nullptr;
      for (float* b : buf)
        if (b != Qc && b != BQ) (R1 ? R2 : R1) = b;
      {
        frpca_ctx::Scope t(h, FRPCA_T_TSMM);
        launch_tsmm(Qc, false, LP, Ns, l, h->W, l, l, LP, R1, LP, nullptr, 0, st);
        launch_tsmm(BQ, false, LP, Ns, l, h->W, l, l, LP, R2, LP, nullptr, 0, st);
      }
      launch_resid_norms(R1, R2, LP, Ns, l, h->d, h->res_tmp, h->res, st);
      check_launch();
      FRPCA_HIP(hipMemcpyAsync(r2.data(), h->res, l * sizeof(double), hipMemcpyDeviceToHost, st));
      FRPCA_HIP(hipMemcpyAsync(theta.data(), h->d, l * sizeof(double), hipMemcpyDeviceToHost, st));
      FRPCA_HIP(hipStreamSynchronize(st));
      // converged when each of the k largest Ritz pairs has ||B w - theta w|| <= tol theta
      // (relative to its own eigenvalue), or <= kResFloor theta_max, the level at which FP32
      // panels stop resolving it; a Ritz value of 0 (a direction the basis lost) never counts
      const double tmax = std::max(theta[l - 1], 0.0);
      if (!(tmax > 0.0)) break;
      bool conv = true;
      double worst = 0.0;
      for (int j = l - k; j < l; ++j) {
        const double rj = std::sqrt(std::max(r2[j], 0.0));
        conv = conv && theta[j] > 0.0 && rj <= std::max(tol * theta[j], kResFloor * tmax);
        worst = std::max(worst, rj / std::max(theta[j], 1e-300 * tmax));
      }
      if (conv) break;
      // stagnation (no 10% gain of the worst relative residual over three steps) ends it too
      hist.push_back(worst);
      if (hist.size() >= 4 && !(worst < 0.9 * hist[hist.size() - 4])) break;
      // Chebyshev filter on the Ritz vectors: damp [0, theta_min] (the unwanted part of the
      // spectrum lies below the block's smallest Ritz value), normalised at theta_max (the scaled
      // three-term recurrence of Zhou and Saad, 2007). Its degree (at most kChebDegree) keeps
      // the growth of the largest Ritz value over the block's smallest, T_d(x_max), and over the
      // k-th largest, T_d(x_max) / T_d(x_k), below 1e5 and 1e4, so no direction of the block
      // sinks under FP32 rounding before the next orthonormalisation. Without a usable interval
      // (theta_min <= 0 after a dropped direction, or no gap) the step is a plain power step.
      float* Xprev = R1;  // Ritz vectors Qc W (the filter's start)
      float* Ycur = R2;
      float* BY = BQ;
      const double bcut = theta[0];
      if (!(bcut > 0.0) || !(tmax > bcut * (1.0 + 1e-12))) {
        apply_B(Xprev, Ycur);
      } else {
        const double e = 0.5 * bcut, c = 0.5 * bcut;
        const double xmax = (tmax - c) / e, xk = (std::max(theta[l - k], 0.0) - c) / e;
        int degree = 1;
        {
          double a0 = 1.0, a1 = xmax, b0 = 1.0, b1 = xk;  // T_0, T_1 at x_max and x_k
          for (int dgr = 2; dgr <= kChebDegree; ++dgr) {
            const double a2 = 2.0 * xmax * a1 - a0, b2 = 2.0 * xk * b1 - b0;
            if (!(std::fabs(a2) <= 1e5) || !(std::fabs(a2) <= 1e4 * std::fabs(b2))) break;
            degree = dgr;
            a0 = a1;
            a1 = a2;
            b0 = b1;
            b1 = b2;
          }
        }
        double sigma = e / (tmax - c);
        const double tau = 2.0 / sigma;
        apply_B(Xprev, BY);
        launch_panel_comb(Ns, l, LP, (float)(sigma / e), BY, (float)(-c * sigma / e), Xprev, 0.f, nullptr, Ycur, st);
        for (int deg = 2; deg <= degree; ++deg) {
          const double sigma_new = 1.0 / (tau - sigma);
          apply_B(Ycur, BY);
          // Y_next = (2 sigma_new / e) (B Y - c Y) - sigma sigma_new X, written over X
          launch_panel_comb(Ns, l, LP, (float)(2.0 * sigma_new / e), BY, (float)(-2.0 * sigma_new * c / e), Ycur,
                            (float)(-sigma * sigma_new), Xprev, Xprev, st);
          std::swap(Xprev, Ycur);
          sigma = sigma_new;
        }
      }
      Qc = Ycur;
      h->orth_cqr2(Qc, BY, Ns, l, LP, nullptr, st);
    }
    // final step as in Alg. 5/6 with the converged basis: Z = (A Q), the eigenpairs of
    // H = Q^T B Q = Z^T Z (already in d, W), U = Z W / sigma and V = Q W for the k largest
    forward(Qc, h->Z);
    launch_final_coeffs(h->d, h->W, l, k, LP, h->rank_tol, h->B1, h->B2, S, h->Skeep, h->ndrop, st);
    float* out_long = a6 ? U : V;
    float* out_short = a6 ? V : U;
    {
      frpca_ctx::Scope t(h, FRPCA_T_TSMM);
      if (a6) launch_tsmm(Qc, false, LP, Ns, l, h->B2, LP, k, k, out_short, k, nullptr, 0, st, nullptr, 0, nullptr, 0, !h->opts.final_f64);
      else launch_tsmm(h->Z, false, LP, Nl, l, h->B1, LP, k, k, out_long, k, nullptr, 0, st, nullptr, 0, nullptr, 0, !h->opts.final_f64);
    }
    if (!h->opts.no_sign_fix) {
      frpca_ctx::Scope t(h, FRPCA_T_SIGN);
      if (a6) launch_sign_fix(V, n, k, h->B1, h->B2, LP, l, h->sign_tmp, st);
      else launch_sign_fix(V, n, k, h->B2, h->B1, LP, l, h->sign_tmp, st);
    }
    {
      frpca_ctx::Scope t(h, FRPCA_T_TSMM);
      if (a6) launch_tsmm(h->Z, false, LP, Nl, l, h->B1, LP, k, k, out_long, k, nullptr, 0, st, nullptr, 0, nullptr, 0, !h->opts.final_f64);
      else launch_tsmm(Qc, false, LP, Ns, l, h->B2, LP, k, k, out_short, k, nullptr, 0, st, nullptr, 0, nullptr, 0, !h->opts.final_f64);
    }
    check_launch();
    h->info.k = k;
    h->info.s = s_oversample;
    h->info.passes = 0;
    if (iters) *iters = it;
  });
}

// Adjoint at the factors (U m x k, S, V n x k), projected on the pattern. With `saved` the
// factors are the last run's, rebuilt from the library's panels; otherwise they are the
// caller's (leading dimension k). Every panel of the adjoint has leading dimension k rounded
// up to 4 with zero pad columns, so the products run on 16-byte rows at any k.
static void adjoint_impl(frpca_ctx* h, int k, const float* Uc, const float* Sc, const float* Vc, const float* dU,
                  const float* dS, const float* dV, float* dval, bool saved) {
  const int64_t m = h->m, n = h->n;
  const int kp = (k + 3) / 4 * 4;
  hipStream_t st = h->stream;
  auto plan = [&](Arena& a, double*& part, double*& J, double*& K, double*& CU, double*& CV, double*& SP,
                  float*& Ui, float*& Vi, float*& L1, float*& R2, float*& dUp, float*& dVp, double*& wpart,
                  float*& ell, float*& corr) {
    part = a.take<double>(gram_partial_bytes(kp) / sizeof(double));
    J = a.take<double>((size_t)kp * kp);
    K = a.take<double>((size_t)kp * kp);
    CU = a.take<double>((size_t)kp * kp);
    CV = a.take<double>((size_t)kp * kp);
    SP = a.take<double>((size_t)kp * kp);
    Ui = a.take<float>((size_t)m * kp);
    Vi = a.take<float>((size_t)n * kp);
    L1 = a.take<float>((size_t)m * kp);
    R2 = a.take<float>((size_t)n * kp);
    dUp = a.take<float>((size_t)m * kp);
    dVp = a.take<float>((size_t)n * kp);
    wpart = h->opts.center ? a.take<double>(wsum_temp_bytes(m) / sizeof(double)) : nullptr;
    ell = h->opts.center ? a.take<float>(2 * kMaxL) : nullptr;
    corr = h->opts.center ? a.take<float>(std::max<int64_t>(n, 1)) : nullptr;
  };
  double *part, *J, *K, *CU, *CV, *SP, *wpart;
  float *Ui, *Vi, *L1, *R2, *dUp, *dVp, *ell, *corr;
  if (!h->bws || h->bws_k < kp) {
    if (h->bws) {
      FRPCA_HIP(hipStreamSynchronize(st));
      FRPCA_HIP(hipFree(h->bws));
      h->bws = nullptr;
      h->bws_bytes = 0;
      h->bws_k = 0;
    }
    Arena probe;
    plan(probe, part, J, K, CU, CV, SP, Ui, Vi, L1, R2, dUp, dVp, wpart, ell, corr);
    if (h->opts.max_workspace && probe.used + h->setup_bytes + h->ws_bytes > h->opts.max_workspace)
      throw Error{FRPCA_ENOMEM, "backward workspace exceeds opts.max_workspace"};
    if (hipMalloc(&h->bws, probe.used) != hipSuccess) {
      (void)hipGetLastError();
      h->bws = nullptr;
      throw Error{FRPCA_ENOMEM, "backward workspace allocation failed"};
    }
    h->bws_bytes = probe.used;
    h->bws_k = kp;
  }
  Arena a;
  a.base = static_cast<char*>(h->bws);
  plan(a, part, J, K, CU, CV, SP, Ui, Vi, L1, R2, dUp, dVp, wpart, ell, corr);

  auto aligned = [](const float* p) { return (reinterpret_cast<uintptr_t>(p) % 16) == 0; };
  // a caller panel (rows x k) as a kp-wide panel: used in place when it already is one
  auto widen = [&](const float* src, int64_t rows, float* buf) -> const float* {
    if (src == nullptr) return nullptr;
    if (kp == k && aligned(src)) return src;
    launch_pad_copy(src, k, rows, k, buf, kp, st);
    return buf;
  };
  const float* U;
  const float* V;
  const float* S;
  {
    frpca_ctx::Scope t(h, FRPCA_T_BWD);
    if (saved) {
      // U = Z B1, V = Q B2 (Alg. 6) or U = Q B2, V = Z B1 (Alg. 5), as the run formed them
      const int LP = h->saved_ld, l = h->saved_l;
      const bool a6 = m >= n;
      launch_tsmm(h->Z, false, LP, h->long_rows(), l, h->B1, LP, k, kp, a6 ? Ui : Vi, kp, nullptr, 0, st);
      launch_tsmm(h->Q, false, LP, h->short_rows(), l, h->B2, LP, k, kp, a6 ? Vi : Ui, kp, nullptr, 0, st);
      U = Ui;
      V = Vi;
      S = h->Skeep;
    } else {
      U = widen(Uc, m, Ui);
      V = widen(Vc, n, Vi);
      S = Sc;
    }
    const float* dUk = widen(dU, m, dUp);
    const float* dVk = widen(dV, n, dVp);
    if (dU) launch_gram(U, false, kp, dUk, kp, m, k, part, J, k, st);
    if (dV) launch_gram(V, false, kp, dVk, kp, n, k, part, K, k, st);
    launch_adjoint_small(J, K, S, dS, k, dU != nullptr, dV != nullptr, CU, CV, SP, st);
    // L1 = U CU + dU SP and R2 = V CV + dV SP, SP diagonal: one pass each, the dU (dV) term
    // added in the product's epilogue; pad columns come out 0
    launch_tsmm(U, false, kp, m, k, CU, k, k, kp, L1, kp, nullptr, 0, st, dUk, kp, dU ? SP : nullptr, k);
    if (dV) launch_tsmm(V, false, kp, n, k, CV, k, k, kp, R2, kp, nullptr, 0, st, dVk, kp, SP, k);
    // centred matrix: dA = (I - 1 1^T / m) G for the dense adjoint G = L1 V^T + U R2^T, so
    // each row of L1 and of U loses its column mean and dval[e] drops corr[c] = l1.V[c] + lU.R2[c]
    if (h->opts.center) {
      launch_wsum(L1, false, kp, m, kp, nullptr, 1.0 / (double)m, wpart, ell, st);
      if (dV) launch_wsum(U, false, kp, m, kp, nullptr, 1.0 / (double)m, wpart, ell + kMaxL, st);
      launch_center_corr(ell, V, ell + kMaxL, dV ? R2 : nullptr, n, k, kp, corr, st);
    }
  }
  {
    frpca_ctx::Scope t(h, FRPCA_T_SDDMM);
    launch_sddmm(h->rp32, h->col, m, kp, L1, V, dV ? U : nullptr, dV ? R2 : nullptr, dval, st,
                 h->opts.center ? corr : nullptr);
  }
  check_launch();
}

int frpca_backward(frpca_t h, const float* dU, const float* dS, const float* dV, float* dval) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(dval != nullptr || h->nnz == 0, FRPCA_EINVAL, "NULL dval");
    FRPCA_CHECK(h->saved_k > 0, FRPCA_ESTATE,
                "frpca_backward needs the factors of a frpca_run on this handle (none since create or "
                "since the last frpca_set_values)");
    adjoint_impl(h, h->saved_k, nullptr, nullptr, nullptr, dU, dS, dV, dval, true);
  });
}

int frpca_adjoint(frpca_t h, int k, const float* U, const float* S, const float* V, const float* dU,
                  const float* dS, const float* dV, float* dval) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    const int64_t m = h->m, n = h->n;
    FRPCA_CHECK(k >= 1 && k <= std::min<int64_t>(std::min(m, n), kMaxL), FRPCA_EINVAL,
                "need 1 <= k <= min(m, n, 128)");
    FRPCA_CHECK(U && S && V && (dval || h->nnz == 0), FRPCA_EINVAL, "NULL factor or output");
    adjoint_impl(h, k, U, S, V, dU, dS, dV, dval, false);
  });
}

int frpca_get_info(frpca_t h, frpca_info* info) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(info != nullptr, FRPCA_EINVAL, "NULL info");
    h->collect_timers();
    if (h->ws) {
      int nd = 0;
      FRPCA_HIP(hipMemcpyAsync(&nd, h->ndrop, sizeof(int), hipMemcpyDeviceToHost, h->stream));
      FRPCA_HIP(hipStreamSynchronize(h->stream));
      h->info.rank_dropped = nd;
    }
    h->info.workspace_bytes = h->setup_bytes + h->ws_bytes + h->bws_bytes + h->ws2_bytes + h->ws3_bytes;
    *info = h->info;
  });
}

int frpca_reset_timers(frpca_t h) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    h->collect_timers();
    for (int i = 0; i < FRPCA_NTIMERS; ++i) {
      h->info.t_ms[i] = 0.0;
      h->info.t_count[i] = 0;
    }
  });
}

const char* frpca_last_error(frpca_t h) { return h ? h->last_error.c_str() : g_last_error.c_str(); }

int frpca_destroy(frpca_t h) {
  delete h;
  return FRPCA_OK;
}

// ------------------------------------------------------------------ step-level entry points
int frpca_gaussian(frpca_t h, uint64_t seed, int64_t rows, int l, int ld, float* out) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(rows >= 0 && l >= 1 && ld >= l && out, FRPCA_EINVAL, "need rows >= 0, 1 <= l <= ld");
    launch_gaussian(seed, rows, l, ld, out, nullptr, h->stream);
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(h->stream));
  });
}

int frpca_spmm(frpca_t h, int trans, int l, const void* in, int in_bf16, int ld_in, void* out, int out_bf16,
               int ld_out) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    // all columns up to the common leading dimension are computed (pads included)
    const int lp = std::min(std::min(ld_in, ld_out), kMaxL) & ~1;
    FRPCA_CHECK(l >= 1 && l <= kMaxL && lp >= l, FRPCA_EINVAL,
                "need 1 <= l <= 128 and leading dimensions >= l (rounded up to even)");
    FRPCA_CHECK(in && out, FRPCA_EINVAL, "NULL panel");
    float* o32 = out_bf16 ? nullptr : static_cast<float*>(out);
    uint16_t* o16 = out_bf16 ? static_cast<uint16_t*>(out) : nullptr;
    if (trans && h->has_bcsc) {
      DeviceTemp part((size_t)h->bhotp.nseg * lp * sizeof(float));
      h->bcsc_product(lp, in, in_bf16 != 0, ld_in, static_cast<float*>(part.p), o32, o16, ld_out, h->stream);
      check_launch();
      FRPCA_HIP(hipStreamSynchronize(h->stream));
      return;
    }
    const MergePlan& p = trans ? h->csc : h->csr;
    launch_spmm(p, lp, in, in_bf16 != 0, ld_in, o32, o16, ld_out, h->stream);
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(h->stream));
  });
}

int frpca_gram(frpca_t h, int64_t rows, int l, const float* X, int ldx, double* G) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(rows >= 0 && l >= 1 && l <= kMaxL && ldx >= l && X && G, FRPCA_EINVAL, "bad Gram arguments");
    DeviceTemp part(gram_partial_bytes(l));
    launch_gram(X, false, ldx, nullptr, 0, rows, l, static_cast<double*>(part.p), G, l, h->stream,
                h->opts.gram_f32 != 0);
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(h->stream));
  });
}

int frpca_eig(frpca_t h, int l, const double* G, double* W, double* d) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(l >= 1 && l <= kMaxL && G && W && d, FRPCA_EINVAL, "bad eig arguments");
    DeviceTemp misc(eig_scratch_bytes());
    launch_eig(G, l, l, d, W, static_cast<double*>(misc.p), h->stream);
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(h->stream));
  });
}

int frpca_eigsvd(frpca_t h, int64_t rows, int l, const float* X, int ldx, float* Q, int ldq, double* S,
                 double tol) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(rows >= l && l >= 1 && l <= kMaxL && ldx >= l && ldq >= l && X && Q && S, FRPCA_EINVAL,
                "bad eigSVD arguments (need rows >= l)");
    if (tol <= 0.0) tol = kInnerTol;
    DeviceTemp part(gram_partial_bytes(l)), misc(4 * kMaxL * kMaxL * sizeof(double)), etmp(eig_scratch_bytes());
    double* G = static_cast<double*>(misc.p);
    double* W = G + kMaxL * kMaxL;
    double* B = W + kMaxL * kMaxL;
    double* d = B + kMaxL * kMaxL;
    hipStream_t st = h->stream;
    launch_gram(X, false, ldx, nullptr, 0, rows, l, static_cast<double*>(part.p), G, l, st, h->opts.gram_f32 != 0);
    launch_eig(G, l, l, d, W, static_cast<double*>(etmp.p), st);
    launch_eigsvd_coeffs(d, W, l, l, tol, B, S, st);
    launch_tsmm(X, false, ldx, rows, l, B, l, l, l, Q, ldq, nullptr, 0, st);
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(st));
  });
}

int frpca_orth(frpca_t h, int64_t rows, int l, const float* X, int ldx, float* Q, int ldq, double* R,
               int* ndropped) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(rows >= l && l >= 1 && l <= kMaxL && ldx >= l && ldq >= l && X && Q, FRPCA_EINVAL,
                "bad orth arguments (need rows >= l)");
    hipStream_t st = h->stream;
    DeviceTemp part(gram_partial_bytes(l)), misc(6 * kMaxL * kMaxL * sizeof(double)), tmp((size_t)rows * ldq * 4),
        nd(256);
    double* G = static_cast<double*>(misc.p);
    double* B1 = G + kMaxL * kMaxL;
    double* B2 = B1 + kMaxL * kMaxL;
    double* R1 = B2 + kMaxL * kMaxL;
    double* R2 = R1 + kMaxL * kMaxL;
    float* T = static_cast<float*>(tmp.p);
    launch_gram(X, false, ldx, nullptr, 0, rows, l, static_cast<double*>(part.p), G, l, st, false);
    launch_chol_inv(G, l, l, kCholTol, B1, l, R1, nullptr, st);
    launch_tsmm(X, false, ldx, rows, l, B1, l, l, ldq, T, ldq, nullptr, 0, st);
    launch_gram(T, false, ldq, nullptr, 0, rows, l, static_cast<double*>(part.p), G, l, st, false);
    launch_chol_inv(G, l, l, kCholTol, B2, l, R2, static_cast<int*>(nd.p), st);
    launch_tsmm(T, false, ldq, rows, l, B2, l, l, ldq, Q, ldq, nullptr, 0, st);
    if (R) launch_small_matmul(R2, R1, l, R, st);
    check_launch();
    int hnd = 0;
    FRPCA_HIP(hipMemcpyAsync(&hnd, nd.p, sizeof(int), hipMemcpyDeviceToHost, st));
    FRPCA_HIP(hipStreamSynchronize(st));
    if (ndropped) *ndropped = hnd;
  });
}

int frpca_jacobi_svd(frpca_t h, int l, const double* R, double* W, double* d) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(l >= 1 && l <= kMaxL && R && W && d, FRPCA_EINVAL, "bad Jacobi SVD arguments");
    launch_jacobi_svd(R, l, l * 2.220446049250313e-16, d, W, h->stream);
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(h->stream));
  });
}

int frpca_pass(frpca_t h, int l, const float* in, float* out, int fused) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(l >= 1 && l <= kMaxL && l <= std::min(h->m, h->n) && in && out, FRPCA_EINVAL,
                "bad pass arguments");
    const int LP = panel_ld(l);
    h->ensure_workspace(LP, h->opts.panel_bf16 ? 1 : 0);
    hipStream_t st = h->stream;
    const bool a6 = h->m >= h->n;
    const MergePlan& Fp = a6 ? h->csr : h->csc;
    const MergePlan& Bp = a6 ? h->csc : h->csr;
    if (fused) {
      launch_fused_pass(Fp.ptr, Fp.idx, Fp.val, Fp.nseg, in, LP, LP, out, LP, h->short_rows(), st);
    } else {
      launch_spmm(Fp, LP, in, false, LP, h->Z, nullptr, LP, st);
      if (a6 && h->has_bcsc) h->bcsc_product(LP, h->Z, false, LP, h->bpart, out, nullptr, LP, st);
      else launch_spmm(Bp, LP, h->Z, false, LP, out, nullptr, LP, st);
    }
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(st));
  });
}

int frpca_lu(frpca_t h, int64_t rows, int l, const float* X, int ldx, float* Q, int ldq, double tol,
             int* ndropped) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(rows >= 1 && l >= 1 && l <= kMaxL && ldx >= l && ldq >= l && X && Q, FRPCA_EINVAL,
                "bad LU arguments");
    if (tol <= 0.0) tol = kInnerTol;
    DeviceTemp tmp(lu_temp_bytes(rows, l)), B(kMaxL * kMaxL * sizeof(double)), nd(256);
    hipStream_t st = h->stream;
    launch_lu_coeffs(X, ldx, rows, l, tol, static_cast<double*>(B.p), l, tmp.p, static_cast<int*>(nd.p), st);
    launch_tsmm(X, false, ldx, rows, l, static_cast<double*>(B.p), l, l, l, Q, ldq, nullptr, 0, st);
    check_launch();
    int hnd = 0;
    FRPCA_HIP(hipMemcpyAsync(&hnd, nd.p, sizeof(int), hipMemcpyDeviceToHost, st));
    FRPCA_HIP(hipStreamSynchronize(st));
    if (ndropped) *ndropped = hnd;
  });
}

int frpca_tsmm(frpca_t h, int64_t rows, int kdim, int c, const float* X, int ldx, const double* B, float* out,
               int ldo) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(rows >= 0 && kdim >= 1 && kdim <= kMaxL && c >= 1 && c <= kMaxL && ldx >= kdim && ldo >= c && X &&
                    B && out,
                FRPCA_EINVAL, "bad TSMM arguments");
    launch_tsmm(X, false, ldx, rows, kdim, B, c, c, c, out, ldo, nullptr, 0, h->stream);
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(h->stream));
  });
}

int frpca_gather_probe(frpca_t h, const float* P, int64_t rows, int ld, int64_t gathers, uint32_t seed,
                       float* out, float* ms, int64_t* rows_read) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(P && out && ms && rows >= 1 && rows <= 0xFFFFFFFFll && ld >= 128 && (ld & 3) == 0 &&
                    (reinterpret_cast<uintptr_t>(P) & 15) == 0 && gathers >= 1 && gathers <= (int64_t)1 << 40,
                FRPCA_EINVAL, "bad gather probe arguments");
    hipEvent_t e0, e1;
    FRPCA_HIP(hipEventCreate(&e0));
    FRPCA_HIP(hipEventCreate(&e1));
    FRPCA_HIP(hipEventRecord(e0, h->stream));
    launch_gather_probe(P, rows, ld, gathers, seed, out, h->stream);
    check_launch();
    FRPCA_HIP(hipEventRecord(e1, h->stream));
    FRPCA_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    FRPCA_HIP(hipEventElapsedTime(&t, e0, e1));
    FRPCA_HIP(hipEventDestroy(e0));
    FRPCA_HIP(hipEventDestroy(e1));
    *ms = t;
    if (rows_read) *rows_read = gather_probe_rows(gathers);
  });
}

int frpca_sddmm(frpca_t h, int w, const float* P1, const float* Q1, const float* P2, const float* Q2,
                float* dval) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(w >= 1 && w <= kMaxL && P1 && Q1 && dval && ((P2 == nullptr) == (Q2 == nullptr)), FRPCA_EINVAL,
                "bad SDDMM arguments");
    launch_sddmm(h->rp32, h->col, h->m, w, P1, Q1, P2, Q2, dval, h->stream);
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(h->stream));
  });
}

int frpca_export_csc(frpca_t h, int64_t* col_ptr, int32_t* row, int32_t* perm) {
  if (!h) return fail(nullptr, Error{FRPCA_EINVAL, "NULL handle"});
  return guarded(h, [&] {
    FRPCA_CHECK(col_ptr && (h->nnz == 0 || (row && perm)), FRPCA_EINVAL, "NULL output");
    hipStream_t st = h->stream;
    widen_kernel<<<(unsigned)((h->n + 1 + 255) / 256), 256, 0, st>>>(h->cp32, h->n + 1, col_ptr);
    if (h->nnz) {
      FRPCA_HIP(hipMemcpyAsync(row, h->row_csc, h->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
      FRPCA_HIP(hipMemcpyAsync(perm, h->perm, h->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    }
    check_launch();
    FRPCA_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free eig
namespace {

// Device scratch of frpca_eig_noalloc: the reflectors, the cluster solves' columns and the
// hand-over state of the three eigensolver kernels. One copy lives on every GPU the library
// runs on, for the life of the process. Host code never passes this name to a kernel (on the
// host it is only a stand-in for the symbol); it uses the address looked up per device below.
constexpr size_t kNoallocScratchBytes = 288 * 1024;
__device__ __align__(256) char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
void* noalloc_scratch() {
  int dev = -1;
  FRPCA_HIP(hipGetDevice(&dev));
  FRPCA_CHECK(dev >= 0 && dev < kMaxDevices, FRPCA_EINVAL, "device index outside the supported range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    FRPCA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    FRPCA_CHECK(p != nullptr, FRPCA_EHIP, "hipGetSymbolAddress returned no address for the eig scratch");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

}  // namespace

extern "C" {

int frpca_eig_noalloc(int l, const double* G, double* W, double* d, void* stream) {
  return guarded(nullptr, [&] {
    FRPCA_CHECK(l >= 1 && l <= kMaxL, FRPCA_EINVAL,
                "l = " + std::to_string(l) + " is outside 1..128, the range the static eig scratch holds");
    FRPCA_CHECK(G && W && d, FRPCA_EINVAL, "NULL G, W or d");
    FRPCA_CHECK(eig_scratch_bytes() <= kNoallocScratchBytes, FRPCA_EHIP,
                "eigensolver scratch larger than the static buffer");
    double* buf = static_cast<double*>(noalloc_scratch());
    launch_eig(G, l, l, d, W, buf, static_cast<hipStream_t>(stream));
    check_launch();
  });
}

}  // extern "C"
