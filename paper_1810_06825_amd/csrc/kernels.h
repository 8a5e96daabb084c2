// Launchers of the gfx950 kernels (internal to the library; host-callable, enqueue only).
#pragma once

#include "common.h"

namespace frpca {

// Rank-1 term subtracted from every finished output row, out[r] -= s[r] v (the centred
// products of k_center.hip); none when v is null, s = 1 when null.
struct SpmmCorr {
  const float* v = nullptr;  // [lp]
  const float* s = nullptr;  // [output rows]
};

// ---------------------------------------------------------------- Gaussian test matrix
// out[r*ld + j] = normal(seed, r*l + j) for j < l, 0 for l <= j < ld; FP32 and/or BF16.
void launch_gaussian(uint64_t seed, int64_t rows, int l, int ld, float* out_f32,
                     uint16_t* out_bf16, hipStream_t st);

// ---------------------------------------------------------------- setup (create)
// flag bits: 1 bad row_ptr ends, 2 decreasing row_ptr, 4 column out of range,
// 8 columns not strictly increasing in a row, 16 non-finite value.
void launch_validate_csr(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                         const int32_t* col, const float* val, int* flag, hipStream_t st);
void launch_ptr_to_i32(const int64_t* p, int64_t count, int32_t* out, hipStream_t st);
void launch_expand_rows(const int32_t* rp, int64_t m, int64_t nnz, int32_t* row_of,
                        hipStream_t st);
// Exclusive scan of count int32 values: out[i] = sum(in[0..i)), out[count] = total.
size_t scan_temp_bytes(int64_t count);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t count, void* temp,
                        hipStream_t st);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the keys. The
// sorted result ends in keys/vals (the *_alt arrays are scratch of the same size).
size_t radix_temp_bytes(int64_t count);
void radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                      int64_t count, int bits, void* temp, hipStream_t st);
// ptr[0..nseg]: ptr[c] = first position of keys (sorted ascending, values < nseg) >= c.
void launch_ptr_from_sorted(const uint32_t* keys, int64_t count, int64_t nseg, int32_t* ptr,
                            hipStream_t st);
void launch_gather_csc(const uint32_t* perm, const int32_t* row_of, const float* val,
                       int64_t nnz, int32_t* row_csc, float* val_csc, hipStream_t st);
void launch_gather_values(const int32_t* perm, const float* val, int64_t nnz, float* out,
                          hipStream_t st);
// Row-blocked order from the column-major mirror (cp, row_csc with rows ascending per column):
// cnt/src[b * hh + h] = length and mirror start of hot column hotcol[h]'s run in row block b
// (blocks of 2^shift rows), cnt/src[nblk * hh + t] = the whole tail column tailcol[t]. After
// an exclusive scan of cnt into bptr, launch_bcsc_copy moves each run (rows and values) to
// bptr[seg]; launch_bcsc_values moves the values alone (after new values reach the mirror).
void launch_bcsc_runs(const int32_t* cp, const int32_t* row_csc, const int32_t* hotcol, const int32_t* tailcol,
                      int64_t hh, int64_t nblk, int64_t ntail, int shift, int32_t* cnt, int32_t* src, hipStream_t st);
void launch_bcsc_copy(const int32_t* bptr, const int32_t* src, int64_t nseg, const int32_t* row_csc,
                      const float* val_csc, int32_t* brow, float* bval, hipStream_t st);
void launch_bcsc_values(const int32_t* bptr, const int32_t* src, int64_t nseg, const float* val_csc, float* bval,
                        hipStream_t st);

// ---------------------------------------------------------------- blocked column order
// (hot columns split by blocks of 2^kBcscRowShift rows; see k_bcsc.hip)
#ifndef FRPCA_BCSC_ROW_SHIFT
#define FRPCA_BCSC_ROW_SHIFT 12
#endif
constexpr int kBcscRowShift = FRPCA_BCSC_ROW_SHIFT;
#ifndef FRPCA_HOT_PER_BLOCK
#define FRPCA_HOT_PER_BLOCK 6
#endif
constexpr int kHotPerBlock = FRPCA_HOT_PER_BLOCK;
void launch_hot_flags(const int32_t* cp, int64_t n, int32_t thresh, int32_t* hot, int32_t* tail, hipStream_t st);
void launch_colmap(const int32_t* hot, const int32_t* hpre, const int32_t* tpre, int64_t n, int32_t* colmap,
                   hipStream_t st);
// segments: nblk * hot_cols hot ones (row block major), then one per tail column
void launch_rebase(const int32_t* ptr, int64_t count, int32_t base, int32_t* out, hipStream_t st);
// X[c] = sum over row blocks of the hot partial rows of c (fixed order), or the tail row of c.
void launch_colmap_inverse(const int32_t* colmap, int64_t n, int32_t* hotcol, int32_t* tailcol, hipStream_t st);
void launch_bcsc_combine(const float* P, int ldp, const int32_t* hotcol, int64_t hot_cols, int64_t nblk, int lp,
                         float* X32, uint16_t* X16, int ldx, hipStream_t st, SpmmCorr corr = {});
// centred products (k_center.hip)
void launch_colmean(const int32_t* cp, const float* val, int64_t n, int64_t m, float* mu, hipStream_t st);
size_t wsum_temp_bytes(int64_t rows);
void launch_wsum(const void* P, bool bf16, int ldp, int64_t rows, int lp, const float* w, double scale, double* part,
                 float* v, hipStream_t st);
void launch_center_corr(const float* a, const float* V, const float* b, const float* R, int64_t n, int k, int ld,
                        float* corr, hipStream_t st);
// dst (rows x ldd) = src (rows x cols, leading dimension lds) with zero columns cols..ldd-1
void launch_pad_copy(const float* src, int lds, int64_t rows, int cols, float* dst, int ldd, hipStream_t st);

// ---------------------------------------------------------------- merge-path products
struct MergePlan {
  const int32_t* ptr = nullptr;   // segment pointers [nseg+1]
  const int32_t* idx = nullptr;   // gathered-row index per nonzero [nnz]
  const float* val = nullptr;     // value per nonzero [nnz]
  int64_t nseg = 0, nnz = 0;
  int64_t nwaves = 0;             // number of merge-path partitions (one wave each)
  int64_t ipw = 0;                // merge items (nonzeros + segment ends) per wave
  int32_t* part_seg = nullptr;    // [nwaves+1] first segment of each partition
  int32_t* part_e = nullptr;      // [nwaves+1] first nonzero of each partition
  int32_t* fix_w0 = nullptr;      // [nwaves] first carrying wave of the segment whose
                                  //   head ends in wave w, or -1
  int sweep = 0;                  // resident waves walk the partitions in narrow rounds
  const int32_t* out_row = nullptr;  // [nseg] output row of each segment (identity when null)
  float* carry = nullptr;         // [nwaves*128] partial sums carried out of each wave
  float* head = nullptr;          // [nwaves*128] partial sums of continued first segments
  int32_t* sweep_ctr = nullptr;   // sweep mode: per-XCD partition counters (8 x 32 ints)
  int64_t in_rows = 0;            // rows of the gathered panel (0: unknown)
};
// Gathered panels larger than this are read with streaming (non-temporal) loads: 8 times the
// 256 MB Infinity Cache, where a random row is almost never found there again. Measured: the
// transpose product's tail part on a 6.6 GB panel 6% faster; on a 512 MB panel (half of it
// cached) streaming loads were 22% slower.
constexpr double kStreamPanelBytes = 2.0 * 1024 * 1024 * 1024;
int64_t merge_items_per_wave(int64_t nseg, int64_t nnz);
#ifndef FRPCA_SWEEP_IPW
#define FRPCA_SWEEP_IPW 384
#endif
constexpr int64_t kSweepItemsPerWave = FRPCA_SWEEP_IPW;  // largest partition of sweep-mode plans
#ifndef FRPCA_SWEEP_PARTS
#define FRPCA_SWEEP_PARTS 256  // sweep partitions per row block (before the ipw clamps)
#endif
#ifndef FRPCA_SWEEP_MIN_IPW
#define FRPCA_SWEEP_MIN_IPW 96
#endif
constexpr int64_t kSweepMinIpw = FRPCA_SWEEP_MIN_IPW;   // smallest partition of sweep-mode plans
void launch_merge_partition(MergePlan& p, hipStream_t st);
void launch_merge_fixplan(MergePlan& p, hipStream_t st);
// out[seg, 0:lp) = sum_{e in seg} val[e] * in[idx[e], 0:lp)  (lp even, <= 128):
// launch_spmm_main writes every segment that ends inside one partition and the carries of
// cut segments; launch_spmm_fixup then completes the cut segments. launch_spmm does both.
void launch_spmm_main(const MergePlan& p, int lp, const void* in, bool in_bf16, int ld_in,
                      float* out_f32, uint16_t* out_bf16, int ld_out, hipStream_t st, SpmmCorr corr = {});
void launch_spmm_fixup(const MergePlan& p, int lp, float* out_f32, uint16_t* out_bf16,
                       int ld_out, hipStream_t st, SpmmCorr corr = {});
void launch_spmm(const MergePlan& p, int lp, const void* in, bool in_bf16, int ld_in,
                 float* out_f32, uint16_t* out_bf16, int ld_out, hipStream_t st, SpmmCorr corr = {});

// ---------------------------------------------------------------- dense kernels
// Gram G = X1^T X2 (l x l, FP64, ld = ldg) of tall panels (rows x l); symmetric when
// X2 == nullptr (X2 = X1). partial: scratch of gram_partial_bytes(). f32_mfma (symmetric
// Gram only): FP32 MFMA with FP32 partial sums over 16 rows, added in FP64 (default: FP64 MFMA).
size_t gram_partial_bytes(int l);
void launch_gram(const void* X1, bool bf16, int ld1, const float* X2, int ld2, int64_t rows,
                 int l, double* partial, double* G, int ldg, hipStream_t st, bool f32_mfma = false);
// out[rows x c_out] = X[rows x kdim] B[kdim x c] (+ y2 diag(d2) when y2 is given); columns
// c..c_out-1 written as 0. FP64 MFMA accumulation, the y2 term added in FP64 before the one
// rounding to FP32; with f32_mfma (FP32 X only), B rounded to FP32 and FP32 MFMA accumulation at
// twice the rate, for well-conditioned B. out (optional) and out_bf16 (optional) receive FP32
// and BF16 results.
void launch_tsmm(const void* X, bool x_bf16, int ldx, int64_t rows, int kdim, const double* B,
                 int ldb, int c, int c_out, float* out, int ldo, uint16_t* out_bf16, int ldo16,
                 hipStream_t st, const float* y2 = nullptr, int ldy2 = 0, const double* d2 = nullptr,
                 int ldd2 = 0, bool f32_mfma = false);

// Symmetric eigendecomposition (G: l x l FP64, ldg): Householder tridiagonalization, then
// relatively robust representations (three launches). d ascending, W l x l row-major
// (column j pairs with d[j]); scratch holds eig_scratch_bytes() of device memory.
size_t eig_scratch_bytes();
void launch_eig(const double* G, int ldg, int l, double* d, double* W, double* scratch, hipStream_t st);
// eigSVD basis coefficients: B[a][j] = W[a][j] / sigma_j (0 if sigma_j <= tol*max), sigma out.
void launch_eigsvd_coeffs(const double* d, const double* W, int l, int ldb, double tol,
                          double* B, double* sigma, hipStream_t st);
// Final Rayleigh-Ritz selection ind = l-1 .. l-k: S[i] = sigma_{l-1-i},
// Blong[a][i] = W[a][l-1-i]/S[i], Bshort[a][i] = W[a][l-1-i]; dropped -> 0. S_keep (optional)
// receives a copy of S.
void launch_final_coeffs(const double* d, const double* W, int l, int k, int ldb,
                         double rank_tol, double* Blong, double* Bshort, float* S, float* S_keep,
                         int* ndropped, hipStream_t st);
// Sign convention on V (rows x k, ld k): sign_i = sign of V's largest-|.| entry of column i.
size_t sign_partial_bytes(int64_t rows, int k);
// Blong and B_other (brows x ldb; B_other may be null) get the same column signs, so factors
// formed from them (U = Z Blong before or after, V = Q B_other again later) inherit them.
void launch_sign_fix(float* V, int64_t rows, int k, double* Blong, double* B_other, int ldb, int brows, void* partial,
                     hipStream_t st);

// LU basis (tournament pivoting) -> coefficient matrix B (l x l, FP64, ldb) with Q = X B.
size_t lu_temp_bytes(int64_t rows, int l);
void launch_lu_coeffs(const float* X, int ldx, int64_t rows, int l, double tol, double* B,
                      int ldb, void* temp, int* ndropped_dev, hipStream_t st);

// ---------------------------------------------------------------- basic rPCA (k_qr.hip)
// Cholesky G = R^T R of an l x l FP64 Gram matrix (ldg) and R^-1 as TSMM coefficients Binv
// (l x ldb, zero padded); a pivot <= tol * G_jj drops column j (zero row of R, zero column
// of R^-1). R (l x l, ld l) and ndrop (device int) are optional outputs.
void launch_chol_inv(const double* G, int ldg, int l, double tol, double* Binv, int ldb, double* R, int* ndrop,
                     hipStream_t st);
// C = A B for l x l FP64 matrices (ld l).
void launch_small_matmul(const double* A, const double* B, int l, double* C, hipStream_t st);
// One-sided Jacobi SVD of R (l x l, ld l): d = sigma^2 ascending, W (l x l row-major) the
// right singular vectors of R paired with d (the layout of launch_eig).
void launch_jacobi_svd(const double* R, int l, double tol, double* d, double* W, hipStream_t st);

// ---------------------------------------------------------------- gather ceiling (k_probe.hip)
// Random 512-byte row reads of P (rows x ld floats, ld >= 128, 16-byte aligned rows) in the
// products' lane shape; gather_probe_rows(g) is the number actually read (g rounded up to a
// multiple of 2048, whole workgroups). out: 64 floats, written only if a sum hits an impossible value.
int64_t gather_probe_rows(int64_t gathers);
void launch_gather_probe(const float* P, int64_t rows, int ld, int64_t gathers, uint32_t seed, float* out,
                         hipStream_t st);

// ---------------------------------------------------------------- eigSVDs (k_cheb.hip)
// out = a X + b Y + c Z elementwise over a rows x ld panel (columns >= cols set to 0);
// Z may be null, out may alias Z.
void launch_panel_comb(int64_t rows, int cols, int ld, float a, const float* X, float b, const float* Y, float c,
                       const float* Z, float* out, hipStream_t st);
// out[j] = || Z[:, j] - theta_j Q[:, j] ||^2 for j < l (FP64, fixed-order reduction).
size_t resid_temp_bytes(int64_t rows);
// G = (G + G^T) / 2 (l x l, ld l) in place.
void launch_symmetrize(double* G, int l, hipStream_t st);
void launch_resid_norms(const float* Q, const float* Z, int ld, int64_t rows, int l, const double* theta,
                        double* temp, double* out, hipStream_t st);

// ---------------------------------------------------------------- fused pass pair (k_fused.hip)
// X (xrows x ldx, zeroed first) = S^T (S Q) for the segment matrix S = (ptr, idx, val) with
// nseg rows: t_r = s_r Q in registers, then atomic adds of s_r^T t_r into X (not bitwise
// repeatable). Q rows and X rows 16-byte aligned, lp a multiple of 4.
void launch_fused_pass(const int32_t* ptr, const int32_t* idx, const float* val, int64_t nseg, const float* Q,
                       int ldq, int lp, float* X, int ldx, int64_t xrows, hipStream_t st);

// ---------------------------------------------------------------- adjoint
// From J = U^T dU, K = V^T dV (k x k, FP64, ld k) and S, dS: coefficient matrices
// CU = M - J S+, CV = -K S+, SP = diag(S+) (k x k, FP64, ld k).
void launch_adjoint_small(const double* J, const double* K, const float* S, const float* dS,
                          int k, bool has_du, bool has_dv, double* CU, double* CV, double* SP,
                          hipStream_t st);
void launch_sddmm(const int32_t* rp, const int32_t* col, int64_t m, int w, const float* P1,
                  const float* Q1, const float* P2, const float* Q2, float* dval, hipStream_t st,
                  const float* corr = nullptr);

}  // namespace frpca
