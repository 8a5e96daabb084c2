/*
 * frpca.h - C interface of the MI355X (gfx950) implementation of fast randomized PCA for
 * sparse data: frPCA (Alg. 5, m <= n) and frPCAt (Alg. 6, m >= n) of Feng, Xie, Song, Yu
 * and Tang, "Fast Randomized PCA for Sparse Data", ACML 2018.
 *
 * Conventions shared by every entry point
 *  - Pointers named as device pointers must address HIP device memory of the current
 *    device; host pointers are plain host memory. The library never takes ownership of a
 *    caller buffer. Dense panels are row-major.
 *  - A CSR matrix is canonical: row_ptr[0] = 0, row_ptr[m] = nnz, non-decreasing row_ptr,
 *    column indices in [0, n) strictly increasing inside each row, finite values,
 *    nnz < 2^31.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). Work is
 *    enqueued on it; calls return before the GPU finishes unless stated otherwise.
 *  - Every entry point returns FRPCA_OK (0) or a negative status. On FRPCA_EINVAL no
 *    output is written. frpca_last_error() describes the most recent failure.
 *  - A handle is not thread-safe; distinct handles may be used from distinct threads.
 */
#ifndef FRPCA_H
#define FRPCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FRPCA_OK 0
#define FRPCA_EINVAL (-1) /* bad argument or malformed CSR                          */
#define FRPCA_ENOMEM (-2) /* device allocation failed or exceeds opts.max_workspace  */
#define FRPCA_EHIP (-3)   /* a HIP runtime call failed                               */
#define FRPCA_ESTATE (-4) /* call not valid in the handle's current state            */

/* Kernel classes timed when opts.timing is set (indices into frpca_info.t_ms). */
#define FRPCA_T_GAUSS 0   /* Gaussian test matrix                                    */
#define FRPCA_T_SPMM_F 1  /* sparse x panel into the long side (A Q in Alg. 6)        */
#define FRPCA_T_SPMM_B 2  /* sparse^T x panel back to the short side (A^T Y, Alg. 6)  */
#define FRPCA_T_GRAM 3    /* X^T X Gram matrix (FP64 MFMA)                          */
#define FRPCA_T_EIG 4     /* symmetric eigendecomposition of the Gram matrix         */
#define FRPCA_T_LU 5      /* LU basis: pivot selection + factor/inverse              */
#define FRPCA_T_TSMM 6    /* tall-skinny panel x small matrix (MFMA)                 */
#define FRPCA_T_SIGN 7    /* output sign convention                                   */
#define FRPCA_T_BWD 8     /* adjoint: cross-Gram, k x k terms, panels                  */
#define FRPCA_T_SDDMM 9   /* adjoint projected onto the sparsity pattern              */
#define FRPCA_T_SPMM_FIX 10 /* merge-path carry fix-up of both products               */
#define FRPCA_T_SPMM_COMB 11 /* row-block partials of the transpose product combined   */
#define FRPCA_T_SPMM_TAIL 12 /* transpose product, columns outside the row-block part  */
#define FRPCA_T_CENTER 13 /* rank-1 terms of the centred products (opts.center)       */
#define FRPCA_T_QR 14     /* Cholesky factors and small SVD of the basic algorithms   */
#define FRPCA_NTIMERS 15

typedef struct frpca_ctx* frpca_t;

/* Options; a zero-initialised struct selects every default. */
typedef struct {
  int panel_bf16;       /* 1: inner-pass panels (the basis fed to the forward product and
                           the long-side panel fed to the back product) are stored in BF16
                           (round to nearest even) with FP32 accumulation; the final pass
                           reads the FP32 basis. 2: the same except in the last inner pass
                           pair (the one before the final eigSVD basis), which stays FP32,
                           so a BF16 rounding only perturbs the starting subspace of a pass
                           pair that follows. 3: only the basis read by the inner forward
                           products is stored in BF16 (the long-side panel stays FP32).
                           4: as 2 for the long-side panel only (the basis stays FP32).
                           0 (default): FP32 panels.                                   */
  int no_sign_fix;      /* 0 (default): flip each (u_i, v_i) so that the largest-|.| entry
                           of v_i is positive (ties: lowest index). 1: leave signs.      */
  double rank_tol;      /* singular values <= rank_tol * sigma_max of the final eigSVD
                           are reported as 0 with zero U/V columns. 0 selects 1e-5.    */
  int timing;           /* 1: time each kernel class with HIP events (frpca_get_info). */
  size_t max_workspace; /* 0: unlimited; else frpca_run fails with FRPCA_ENOMEM if its
                           device workspace would exceed this many bytes.             */
  int center;           /* 1: principal components of the column-centred matrix
                           A - 1 mu^T (mu = column means of A), the PCA of data with rows
                           as samples (Section 1 assumes centred data), without forming it:
                           each product with A or A^T gets its rank-1 term; the column
                           means follow frpca_set_values; frpca_backward then returns the
                           gradient with respect to A's stored values through the
                           centring. 0 (default): A itself.                            */
  int gram_f32;         /* 1: the Gram matrices of eigSVD (Alg. 2) use the FP32 matrix
                           cores: FP32 partial sums over 16 rows, added in FP64. Relative
                           error of sigma_k up to about 8 u32 (sigma_1/sigma_k)^2
                           (u32 = 2^-24: half the 16-row sum times unit roundoff).
                           0 (default): FP64 matrix cores on the FP32 panels, each product
                           exact and only the FP64 sums rounded.                      */
  int fused_pass;       /* 1: each inner pass pair of frpca_run (A^T (A Q) in Alg. 6,
                           A (A^T Q) in Alg. 5) runs as one sweep: t_r = a_r Q is formed in
                           registers and a_r^T t_r is added into the short-side panel with
                           floating-point atomics, so the long-side panel is never stored.
                           The order of the atomic adds varies, so results are not bitwise
                           repeatable; not with center or panel_bf16. 0 (default): the two
                           deterministic products of the merge-path plans.            */
  int final_f64;        /* 1: the final products that form the outputs (U and V from the
                           last panels and the l x k coefficient matrices) accumulate on
                           the FP64 matrix cores. 0 (default): on the FP32 matrix cores at
                           twice the rate, the coefficients rounded to FP32; their
                           matrices are orthogonal or scaled by 1/sigma, so the outputs move
                           by about one FP32 rounding per term (orthonormality ~1e-7). */
} frpca_opts;

typedef struct {
  int64_t m, n, nnz;
  int orientation;        /* 6: Alg. 6 (m >= n); 5: Alg. 5 (m < n)                    */
  int k, s, passes;       /* of the last frpca_run                                    */
  int rank_dropped;       /* output singular values set to 0 by rank_tol (last run)   */
  size_t workspace_bytes; /* device memory currently held by the handle               */
  double create_ms;       /* wall time of frpca_create (validation + CSC mirror)       */
  int64_t hot_cols;       /* columns whose A^T products run in row blocks (0: none)   */
  int64_t row_blocks;     /* row blocks of 4096 rows used for them                    */
  int64_t hot_nnz;        /* nonzeros in those columns                                */
  double t_ms[FRPCA_NTIMERS];   /* accumulated GPU time per kernel class (opts.timing) */
  int64_t t_count[FRPCA_NTIMERS]; /* number of timed launches per class                */
} frpca_info;

/*
 * frpca_create - bind a CSR matrix and build its column-major mirror.
 * Defines: the input A of Alg. 5/6 (m x n sparse). The paper avoids forming A^T because the
 * sparse storage makes it awkward (Section 3.2); here a column-major copy of the pattern
 * (col_ptr, row indices, permutation into CSR order, values) is built once on the GPU by a
 * stable sort of the nonzeros by column, so both products run without atomics.
 * row_ptr (int64[m+1]), col (int32[nnz]), val (float[nnz]) are device pointers, borrowed:
 * they must stay allocated and unchanged until frpca_destroy (after changing the values,
 * call frpca_set_values). Validates the CSR on the device and synchronises `stream` once.
 * *out receives the handle (NULL on failure). Errors: EINVAL (shape, malformed CSR,
 * non-finite value), ENOMEM, EHIP.
 */
int frpca_create(frpca_t* out, int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                 const int32_t* col, const float* val, const frpca_opts* opts, void* stream);

/* frpca_set_values - the CSR values changed (same pattern); refresh the mirror's values.
 * val: device float[nnz] (borrowed as in frpca_create). Asynchronous. */
int frpca_set_values(frpca_t h, const float* val);

/* frpca_set_stream - enqueue subsequent work of h on `stream`. When the stream changes, work
 * on the new stream starts after everything already queued on the old one (an event). */
int frpca_set_stream(frpca_t h, void* stream);

/*
 * frpca_run - rank-k truncated SVD A ~ U diag(S) V^T by Alg. 6 (m >= n) or Alg. 5 (m < n).
 * Defines: Alg. 5 / Alg. 6 (Section 3.3) with pass parameter q = p_passes >= 2 (number of
 * passes over A), oversampling s = s_oversample >= 0, l = k + s <= min(m, n), l <= 128;
 * inner LU bases (Lemma 3, eq. 8) and eigSVD bases (Alg. 2); the Gaussian test matrix is
 * drawn from Philox4x32-10 with key `seed` (element [r, j] of the rows x l draw is normal
 * number r*l + j: Box-Muller in FP64 on words (x0,x1), (x2,x3) of block t/4, rounded to
 * FP32). Outputs (device, row-major, caller-allocated): U float[m*k], S float[k]
 * (descending), V float[n*k]. Sign and rank conventions: see frpca_opts.
 * Asynchronous; the handle's workspace is (re)allocated on the first call for a larger l.
 * Errors: EINVAL (k < 1, s < 0, k+s > min(m,n), k+s > 128, p_passes < 2), ENOMEM, EHIP.
 */
int frpca_run(frpca_t h, int k, int p_passes, int s_oversample, uint64_t seed, float* U,
              float* S, float* V);

/*
 * frpca_run_basic - rank-k truncated SVD by the basic randomized algorithm that frPCA
 * accelerates: Alg. 1 (basic rPCA, Section 2.2; alg = 1) or Alg. 4 (basic rPCAt, Section
 * 3.2; alg = 4), for any shape of A, with p_power >= 0 power steps (2 p_power + 2 passes
 * over A). Every product with A or A^T is followed by orth(), here CholeskyQR2 (FP64 Gram on
 * the matrix cores, FP64 Cholesky with a rank guard, Q = X R^-1, twice), which by Lemma 2
 * gives the algorithm the result of the paper's Householder QR; the final svd(B) is the
 * CholeskyQR2 factor R of B^T followed by a one-sided Jacobi SVD of R in FP64. Gaussian
 * matrix: Alg. 1 draws Omega as n x l, Alg. 4 draws its l x m Omega stored as m x l (element
 * [r, j] = normal(seed, r*l + j), the draws of frpca_run for odd / even q), so by Theorems 1
 * and 2 the result equals frpca_run with q = 2 p_power + 2 on the matching orientation (Alg. 5
 * from Alg. 1 when m < n, Alg. 6 from Alg. 4 when m >= n). Outputs, rank and sign conventions
 * as frpca_run. frpca_backward does not apply to this path (ESTATE afterwards). The first
 * call allocates a second long-side panel in the handle's workspace.
 * Errors: EINVAL (k < 1, s < 0, k+s > min(m,n), k+s > 128, p_power < 0, alg not 1 or 4),
 * ENOMEM, EHIP.
 */
int frpca_run_basic(frpca_t h, int k, int p_power, int s_oversample, uint64_t seed, int alg, float* U,
                    float* S, float* V);

/*
 * frpca_eigsvds - rank-k truncated SVD by eigSVDs (Alg. 3, Section 3.1): the k largest
 * eigenpairs of B = A^T A (m >= n; A A^T when m < n, the smaller Gram matrix), S = their
 * square roots, V the eigenvectors, U = A V diag(1/S). The eigenpairs come from a block
 * subspace iteration on B with Rayleigh-Ritz steps, as eigs(B, k) would compute them: a
 * block of l = k + s_oversample >= k columns starts from a Gaussian matrix (normal(seed,
 * r*l + j) as in frpca_run) orthonormalised by CholeskyQR2; each step applies a Chebyshev
 * filter of degree 8 that damps the spectrum below the block's smallest Ritz value,
 * re-orthonormalises, and takes the Ritz pairs of Q^T B Q; it stops when every one of the k
 * largest Ritz pairs has residual ||B w - theta w|| <= tol * theta_max (tol <= 0 selects
 * 1e-6) or after max_iter Rayleigh-Ritz steps. B is applied as A^T (A P), never formed.
 * Outputs, rank and sign conventions as frpca_run; *iters (host int, may be NULL) receives
 * the number of Rayleigh-Ritz steps. The first call allocates two more short-side panels.
 * frpca_backward does not apply (ESTATE afterwards). Errors: EINVAL (k < 1, s < 0,
 * k+s > min(m,n), k+s > 128, max_iter < 1), ENOMEM, EHIP.
 */
int frpca_eigsvds(frpca_t h, int k, int s_oversample, uint64_t seed, double tol, int max_iter, float* U,
                  float* S, float* V, int* iters);

/*
 * frpca_backward - dL/d(values of A) from dL/dU, dL/dS, dL/dV of the handle's last frpca_run,
 * through the truncated-SVD adjoint projected onto the sparsity pattern (not part of the
 * paper; the standard SVD reverse-mode rule): with J = U^T dU, K = V^T dV (FP64),
 * F_ij = 1/(s_j^2 - s_i^2) (i != j, 0 where |s_j^2 - s_i^2| <= 1e-12 s_1^2),
 * S+ = diag(1/s_i or 0),
 *   M = (F o (J - J^T)) S + diag(dS) + S (F o (K - K^T)),
 *   dA = U M V^T + (dU - U J) S+ V^T + U S+ (dV - V K)^T,
 * and dval[e] = dA[row(e), col(e)] in CSR order (with opts.center, the gradient with
 * respect to A's stored values through the centring).
 * The factors U, S, V are those the last frpca_run computed: the library keeps what it needs
 * to rebuild them (the run's long-side panel, short-side basis, final coefficients with the
 * sign convention, and S), so the caller's output buffers may be reused or freed.
 * dU (device float[m*k], row-major), dS (float[k]), dV (float[n*k]) may each be NULL (zero);
 * k is the last run's. dval: device float[nnz]. Asynchronous.
 * Errors: ESTATE (no frpca_run since frpca_create, or frpca_set_values since the last run,
 * or the last run failed), EINVAL (NULL dval with nnz > 0), ENOMEM, EHIP.
 */
int frpca_backward(frpca_t h, const float* dU, const float* dS, const float* dV, float* dval);

/* frpca_get_info - sizes, orientation, last run's parameters and timers (host struct).
 * Synchronises the handle's stream when timing is enabled. */
int frpca_get_info(frpca_t h, frpca_info* info);

/* frpca_reset_timers - zero the accumulated kernel timers. */
int frpca_reset_timers(frpca_t h);

/* frpca_last_error - text of the most recent failure on h (h = NULL: the calling thread's
 * most recent failure outside a handle). Valid until the next call on the same handle. */
const char* frpca_last_error(frpca_t h);

/* frpca_destroy - free all device memory held by h (synchronises its stream). */
int frpca_destroy(frpca_t h);

/* ------------------------------------------------------------------------------------
 * Step-level entry points: one step of the path each, for tests and composition. They
 * use the handle's stream and scratch memory, synchronise before returning, and follow
 * the same numerical definitions as frpca_run. Panels: `l` columns, leading dimension
 * `ld` >= l (elements); BF16 panels are uint16 bit patterns.
 * ------------------------------------------------------------------------------------ */

/* Gaussian test matrix (Alg. 5/6 "randn"): out[r*ld + j] = normal(seed, r*l + j) for
 * r < rows, j < l; columns l..ld-1 are set to 0. out: device float[rows*ld]. */
int frpca_gaussian(frpca_t h, uint64_t seed, int64_t rows, int l, int ld, float* out);

/* Sparse x panel (the products of Alg. 5/6): trans = 0: out = A in (in: n x l, out: m x l);
 * trans = 1: out = A^T in (in: m x l, out: n x l). FP32 accumulation; in_bf16 / out_bf16
 * select BF16 panels. All columns below min(ld_in, ld_out, 128) rounded down to even are
 * computed, so zero pad columns of `in` give zero pad columns of `out`. */
int frpca_spmm(frpca_t h, int trans, int l, const void* in, int in_bf16, int ld_in, void* out,
               int out_bf16, int ld_out);

/* Gram matrix of a tall panel (Alg. 2 step 1): G = X^T X, X: device float[rows*ldx]
 * (l columns), G: device double[l*l] row-major, accumulated in FP64 on MFMA (FP32 MFMA
 * sums over 16 rows, added in FP64, when the handle was created with opts.gram_f32). */
int frpca_gram(frpca_t h, int64_t rows, int l, const float* X, int ldx, double* G);

/* Symmetric eigendecomposition (Alg. 2 step 2) in FP64 (Householder tridiagonalization,
 * then bisection and twisted factorizations on a positive definite L D L^T representation):
 * G (device double[l*l], symmetric) = W diag(d) W^T with d ascending (device double[l])
 * and orthonormal W (device double[l*l] row-major, column j pairs with d[j]). l <= 128.
 * Allocates and frees a device scratch buffer of about 266 KiB per call. */
int frpca_eig(frpca_t h, int l, const double* G, double* W, double* d);

/* frpca_eig_noalloc - the decomposition of frpca_eig without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same kernels and results as frpca_eig (bitwise). Needs no handle:
 * the work is enqueued on `stream` (hipStream_t as void*, NULL = default stream) and the call
 * returns without synchronising. Its scratch is a static device buffer of 288 KiB that every
 * GPU the library runs on holds until the process ends (its address is looked up on the
 * first call on each device). All calls on one GPU share that buffer: calls whose work
 * overlaps on one GPU (concurrent streams, or threads) race and must be serialised by the
 * caller; consecutive calls on one stream are safe. G, W, d: device pointers as in frpca_eig,
 * 1 <= l <= 128. Errors: EINVAL (l outside 1..128, NULL pointer), EHIP; the message goes to
 * frpca_last_error(NULL). */
int frpca_eig_noalloc(int l, const double* G, double* W, double* d, void* stream);

/* eigSVD basis (Alg. 2): Q = X V diag(1/S) with S ascending; S_j <= tol * max(S) gives a
 * zero column (tol <= 0 selects 1e-12). The Gram follows opts.gram_f32 as frpca_gram.
 * X, Q: device float panels (rows x l), S: device double[l] (ascending, zeroed where
 * dropped). */
int frpca_eigsvd(frpca_t h, int64_t rows, int l, const float* X, int ldx, float* Q, int ldq,
                 double* S, double tol);

/* orth() of the basic algorithms: Q = X R^-1 with R the CholeskyQR2 factor of X (rows x l,
 * rows >= l); a column whose Cholesky pivot is <= 1e-13 of its squared norm in either pass is
 * zero in Q (*ndropped, host int, counts them). R (device double[l*l], upper triangular, may
 * be NULL) receives R2 R1. */
int frpca_orth(frpca_t h, int64_t rows, int l, const float* X, int ldx, float* Q, int ldq, double* R,
               int* ndropped);

/* SVD of a small square matrix by one-sided Jacobi in FP64 (the svd(B) step of the basic
 * algorithms, applied to the triangular factor of B^T): R (device double[l*l], row-major)
 * = U_R diag(sqrt(d)) W^T with d (device double[l]) ascending and W (device double[l*l],
 * row-major, column j paired with d[j]) orthonormal; l <= 128. */
int frpca_jacobi_svd(frpca_t h, int l, const double* R, double* W, double* d);

/* One inner pass pair (Section 3.3): out = A^T (A in) when m >= n, A (A^T in) when m < n,
 * for short-side panels in/out (device float, min(m,n) x ld, ld = l rounded up to 32,
 * l <= 128; pad columns of in must be 0, those of out are 0). fused = 0: the two merge-path
 * products through the handle's long-side workspace (deterministic); fused = 1: the one-sweep
 * form of opts.fused_pass (atomic adds). */
int frpca_pass(frpca_t h, int l, const float* in, float* out, int fused);

/* LU basis (Lemma 3, eq. 8): Q = P^T L of P X = L U with pivots chosen by tournament
 * pivoting (partial pivoting inside each node); pivot rows of Q form a unit lower-triangular
 * block. A column whose best remaining pivot is <= tol * max|X| is zero in Q (tol <= 0
 * selects 1e-12). *ndropped (host int) receives the number of zero columns. */
int frpca_lu(frpca_t h, int64_t rows, int l, const float* X, int ldx, float* Q, int ldq,
             double tol, int* ndropped);

/* Tall-skinny product out = X B (rows x c), X: device float[rows*ldx] (kdim columns),
 * B: device double[kdim*c] row-major, FP64 accumulation on MFMA, out: device float. */
int frpca_tsmm(frpca_t h, int64_t rows, int kdim, int c, const float* X, int ldx,
               const double* B, float* out, int ldo);

/* Sampled dense-dense product on the sparsity pattern (the adjoint's projection):
 * dval[e] = sum_i P1[r,i] Q1[c,i] + sum_i P2[r,i] Q2[c,i] for nonzero e = (r, c), CSR
 * order; P1, P2: device float[m*w] (ld w), Q1, Q2: device float[n*w]; P2/Q2 may be NULL. */
int frpca_sddmm(frpca_t h, int w, const float* P1, const float* Q1, const float* P2,
                const float* Q2, float* dval);

/* The adjoint of frpca_backward at caller-given factors: U (device float[m*k]), S (float[k],
 * descending, as frpca_run returns them), V (float[n*k]), 1 <= k <= min(m, n, 128); dU, dS, dV
 * may be NULL. A pure function of its arguments (it neither needs nor uses the last run).
 * Asynchronous. Errors: EINVAL, ENOMEM, EHIP. */
int frpca_adjoint(frpca_t h, int k, const float* U, const float* S, const float* V, const float* dU,
                  const float* dS, const float* dV, float* dval);

/* Copy of the column-major mirror built by frpca_create: col_ptr int64[n+1], row
 * int32[nnz], perm int32[nnz] (CSR position of each column-major nonzero). Device ptrs. */
int frpca_export_csc(frpca_t h, int64_t* col_ptr, int32_t* row, int32_t* perm);

/* Measurement helper (not a step of the method): `gathers` random 512-byte row reads of P
 * (device float[rows*ld], ld >= 128 and a multiple of 4, 16-byte aligned), two rows per wave
 * instruction as in the sparse products, on the handle's stream; *ms (host) receives the
 * kernel's time from HIP events and *rows_read (host, optional) the number of rows read
 * (gathers rounded up to whole workgroups of 2048). out: device float[64], scratch the kernel may
 * write. Synchronous. The rate rows_read * 512 B / ms is the ceiling of the products' gathers
 * beside the streaming peak. Errors: EINVAL, EHIP. */
int frpca_gather_probe(frpca_t h, const float* P, int64_t rows, int ld, int64_t gathers, uint32_t seed,
                       float* out, float* ms, int64_t* rows_read);

#ifdef __cplusplus
}
#endif
#endif /* FRPCA_H */
