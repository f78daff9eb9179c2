/*
 * wprod.h - C ABI of the MI355X (gfx950) w-product library, libwprod.so.
 *
 * The w-product of Panchal & Behera (arXiv 2601.08228) multiplies third-order
 * tensors through a lazy lifting wavelet transform along mode 3 (Sec. II-A,
 * Eq. (1)), slice-wise matrix products of the coefficients (the face-product
 * of Def. 2.1) and the inverse transform (Alg. 1); the w-svd replaces the
 * products by per-slice truncated SVDs (Alg. 2, Thm 2.5).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Memory.  Every tensor pointer is a DEVICE pointer on the calling thread's
 *   current HIP device, allocated and owned by the caller.  The library
 *   allocates no device memory; where scratch is needed the caller passes a
 *   workspace whose size a *_workspace() query returns.  Its only state is
 *   the fixed device scratch of w_product_noalloc (and, per device, that
 *   array's address and a kernel attribute, set on first use).
 * Layout.  A tensor X in R^{n1 x n2 x p} is p contiguous row-major n1 x n2
 *   frontal slices: X[i, j, k] (0-based) lives at element k*n1*n2 + i*n2 + j
 *   (a C-contiguous array of shape (p, n1, n2)).  A coefficient tensor has
 *   the same shape with its slices in the order of Eq. (1): s_L, d_L,
 *   d_{L-1}, ..., d_1, where with m = p / 2^L, s_L occupies slices [0, m) and
 *   d_j occupies slices [p / 2^j, p / 2^(j-1)).
 * Transform.  The lazy lifting of Sec. II-A (P_j = I, U_j = I/2): each level
 *   splits the smooth sequence into pairs (first, second) = (slice 2q, slice
 *   2q+1), d = first - second, s = second + d/2.  p must be a positive
 *   multiple of 2^L; 0 <= L <= 10 (L = 0 is the identity transform).
 * Types.  WP_F64 (double) or WP_F32 (float) elements.  Split-precision
 *   coefficients are two arrays of bfloat16 bit patterns (uint16_t) of the
 *   same shape: hi = bf16_rne(x), lo = bf16_rne(x - hi).
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Every entry
 *   point only enqueues work on it and returns without synchronising; results
 *   are ready when the stream reaches that point.
 * Errors.  Arguments are validated before any HIP call; on an error nothing is
 *   launched, no output is touched, and a negative wp_status is returned.
 *   NaN/Inf inputs are not screened and propagate.  Outputs must not overlap
 *   inputs or each other (WP_EALIAS).  Sizes: every dimension >= 1 and each
 *   tensor below 2^40 elements.
 */
#ifndef WPROD_H
#define WPROD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int wp_status;
#define WP_OK           0
#define WP_EINVAL      -1   /* bad size, level, rank or flag                    */
#define WP_ENULL       -2   /* required pointer is NULL                          */
#define WP_EALIAS      -3   /* an output overlaps an input or another output     */
#define WP_EDTYPE      -4   /* unknown dtype, or GEMM mode not valid for dtype   */
#define WP_EWORKSPACE  -5   /* workspace smaller than the *_workspace() query    */
#define WP_ELAUNCH     -6   /* a HIP launch or runtime call failed               */
#define WP_ENOCONV     -7   /* reported by callers when a Jacobi slice did not converge */
#define WP_ESCRATCH    -8   /* w_product_noalloc: the call needs more than its fixed scratch */

#define WP_F64 0
#define WP_F32 1

#define WP_GEMM_NATIVE 0    /* F64 data on FP64 MFMA, F32 data on FP32 MFMA      */
#define WP_GEMM_BF16   1    /* F32 data, products of bf16 hi parts, FP32 accumulation */
#define WP_GEMM_BF16X3 2    /* F32 data, hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulation */

/* Human-readable name of a status code (static string, never NULL). */
const char* w_status_string(wp_status s);

/* Library ABI version (major*10000 + minor*100 + patch). */
int w_version(void);

/* ---- Transforms (Sec. II-A) -------------------------------------------------
 * In: x or coefficients, (p, n1, n2) of `dtype`.  Out: same shape and dtype.
 */

/* Forward lifting W_[L] along mode 3, Eq. (1) / Alg. 1 forward steps:
 * x (spatial) -> xhat (coefficients, Eq. (1) order). */
wp_status w_transform(const void* x, void* xhat, int64_t n1, int64_t n2, int64_t p,
                      int L, int dtype, void* stream);

/* Inverse lifting W_[L]^{-1}, Eq. (3) / Alg. 1 inverse steps: xhat -> x. */
wp_status w_itransform(const void* xhat, void* x, int64_t n1, int64_t n2, int64_t p,
                       int L, int dtype, void* stream);

/* Transpose W_[L]^T (adjoint of w_transform, derived from its level steps):
 * coefficient-space g -> spatial out.  Used by the reverse-mode derivative. */
wp_status w_transform_adj(const void* g, void* out, int64_t n1, int64_t n2, int64_t p,
                          int L, int dtype, void* stream);

/* Transpose of the inverse, W_[L]^{-T}: spatial g -> coefficient-space out. */
wp_status w_itransform_adj(const void* g, void* out, int64_t n1, int64_t n2, int64_t p,
                           int L, int dtype, void* stream);

/* w_transform of float data with a split-precision epilogue: writes
 * hi = bf16_rne(xhat) and lo = bf16_rne(xhat - hi) (lo may be NULL: hi only). */
wp_status w_transform_split(const float* x, uint16_t* xhat_hi, uint16_t* xhat_lo,
                            int64_t n1, int64_t n2, int64_t p, int L, void* stream);

/* w_itransform_adj of float data with the same split-precision epilogue. */
wp_status w_itransform_adj_split(const float* g, uint16_t* out_hi, uint16_t* out_lo,
                                 int64_t n1, int64_t n2, int64_t p, int L, void* stream);

/* ---- Lifting with chosen predict and update operators (Sec. II-A; Remark 3.1)
 * Level j of W_[L] = W_L ... W_1 splits the current smooth sequence of each
 * mode-3 tube (length l = p / 2^(j-1)) into pairs; o[m] is the first and e[m]
 * the second entry of pair m (the odd and even entries of Alg. 1, whose
 * indices are 1-based), m = 0 .. l/2 - 1, and
 *   d_j = o - P_j e,   s_j = e + U_j d_j,
 *   (P_j e)[m] = sum_t predict_j[t] e[clamp(m + t - 2)], U_j likewise on d_j,
 * indices clamped to [0, l/2 - 1] (the sequence extended by its end values).
 * The inverse undoes the steps in reverse (e = s - U d, o = d + P e).
 * taps: host array of L * 2 * WP_TAPS doubles, level j's predict stencil at
 *   taps[((j-1)*2 + 0)*WP_TAPS + t], its update stencil at
 *   taps[((j-1)*2 + 1)*WP_TAPS + t], tap t at offset t - 2; copied at the
 *   call; every tap finite (WP_EINVAL otherwise); may be NULL when L = 0.
 * predict = {0,0,1,0,0} and update = {0,0,0.5,0,0} at every level give the
 * lazy transform of w_transform (same results, up to rounding order).
 * Limit: p * 16 * element size <= 128 KiB (p <= 1024 for WP_F64, 2048 for
 * WP_F32): a workgroup holds whole tubes in LDS.
 */
#define WP_TAPS 5
#define WP_LIFT_FORWARD 0   /* W_[L]:      x -> coefficients (Eq. (1) order)    */
#define WP_LIFT_INVERSE 1   /* W_[L]^{-1}: coefficients -> x                    */
#define WP_LIFT_ADJ     2   /* W_[L]^T:    coefficient-space g -> spatial       */
#define WP_LIFT_IADJ    3   /* W_[L]^{-T}: spatial g -> coefficient space       */

/* One pass of the scheme (kind WP_LIFT_*) over (p, n1, n2) data; in and out
 * must not overlap. */
wp_status w_transform_scheme(const void* in, void* out, int64_t n1, int64_t n2, int64_t p,
                             int L, const double* taps, int kind, int dtype, void* stream);

/* WP_LIFT_FORWARD or WP_LIFT_IADJ pass of float data with the split-precision
 * epilogue of w_transform_split (bf16 hi, and the bf16 residual lo unless
 * out_lo is NULL). */
wp_status w_transform_scheme_split(const float* in, uint16_t* out_hi, uint16_t* out_lo,
                                   int64_t n1, int64_t n2, int64_t p, int L,
                                   const double* taps, int kind, void* stream);

/* w-product (Def. 2.1) under a scheme: W^{-1}( W(op A) Delta W(op B) ), all
 * arguments as for w_product; ws must hold w_product_scheme_workspace(...)
 * bytes.  BF16 modes split the scheme's coefficients like w_product. */
wp_status w_product_scheme(const void* a, const void* b, void* c,
                           int64_t n1, int64_t n2, int64_t n3, int64_t p, int L,
                           const double* taps, int trans_a, int trans_b, int dtype, int gemm,
                           void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for w_product_scheme (0 on invalid arguments). */
size_t w_product_scheme_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int L,
                                  int dtype, int gemm);

/* ---- Face-product (Def. 2.1, Alg. 1 middle part) ----------------------------
 * Ch[k] = op(Ah[k]) * op(Bh[k]) for k = 0..p-1, with op(X) = X or X^T per
 * slice (Def. 2.2).  op(Ah[k]) is n1 x n2, op(Bh[k]) is n2 x n3, Ch is
 * (p, n1, n3).  Stored shapes: Ah (p, n1, n2), or (p, n2, n1) if trans_a;
 * Bh (p, n2, n3), or (p, n3, n2) if trans_b.  Transposing before or after the
 * transform is the same (Thm 2.1), so the flags apply to spatial operands too.
 */

/* Native precision: WP_F64 on FP64 MFMA, WP_F32 on FP32 MFMA (FP32 accumulation). */
wp_status w_face_product(const void* ah, const void* bh, void* ch,
                         int64_t n1, int64_t n2, int64_t n3, int64_t p,
                         int trans_a, int trans_b, int dtype, void* stream);

/* Split precision on BF16 MFMA with FP32 accumulation.  gemm = WP_GEMM_BF16
 * uses a_hi*b_hi only (a_lo, b_lo may be NULL); WP_GEMM_BF16X3 adds a_hi*b_lo
 * + a_lo*b_hi (all four arrays required).  Output ch is float. */
wp_status w_face_product_split(const uint16_t* a_hi, const uint16_t* a_lo,
                               const uint16_t* b_hi, const uint16_t* b_lo, float* ch,
                               int64_t n1, int64_t n2, int64_t n3, int64_t p,
                               int trans_a, int trans_b, int gemm, void* stream);

/* One call for every arithmetic: gemm = WP_GEMM_NATIVE is w_face_product
 * (ws may be NULL); WP_GEMM_BF16 / WP_GEMM_BF16X3 (float ah, bh, ch) first
 * split both operands into bf16 hi / lo planes in ws (hi = bf16_rne(x),
 * lo = bf16_rne(x - hi)), then run w_face_product_split.  ws (device, caller
 * owned, any alignment) must hold w_face_product_workspace(...) bytes
 * (WP_EWORKSPACE otherwise) and must not overlap ah, bh or ch (WP_EALIAS). */
wp_status w_face_product_gemm(const void* ah, const void* bh, void* ch,
                              int64_t n1, int64_t n2, int64_t n3, int64_t p,
                              int trans_a, int trans_b, int dtype, int gemm,
                              void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for w_face_product_gemm: 0 for WP_GEMM_NATIVE (none needed)
 * and on invalid arguments. */
size_t w_face_product_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p,
                                int dtype, int gemm);

/* ---- w-product (Def. 2.1, Alg. 1) ------------------------------------------
 * C = op(A) *_w op(B) = W^{-1}( W(op A) Delta W(op B) ); C is (p, n1, n3).
 * gemm selects the face-product arithmetic (WP_GEMM_*; BF16 modes need
 * WP_F32).  ws must hold w_product_workspace(...) bytes (256-byte aligned
 * pointer recommended; any alignment is accepted).
 */
wp_status w_product(const void* a, const void* b, void* c,
                    int64_t n1, int64_t n2, int64_t n3, int64_t p, int L,
                    int trans_a, int trans_b, int dtype, int gemm,
                    void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for w_product (0 on invalid arguments). */
size_t w_product_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int L,
                           int dtype, int gemm);

/* w_product for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and results as w_product, with the workspace taken from a fixed
 * device array inside the library instead of a caller buffer.  The caller
 * still passes (and owns) a, b and c.  The array holds
 * w_product_noalloc_scratch_bytes() = 128 MiB; a call whose
 * w_product_workspace(...) is larger returns WP_ESCRATCH before any HIP call.
 * Each device the library runs on holds its own array until the process ends
 * (its address is looked up on the first call on that device, with that device
 * current).  No call allocates or frees memory.  Every call on one device
 * shares that device's array and leaves its contents behind (nothing in it
 * needs to start at zero): calls that overlap on one device (on different
 * streams, or from different host threads) race and must be ordered by the
 * caller. */
wp_status w_product_noalloc(const void* a, const void* b, void* c,
                            int64_t n1, int64_t n2, int64_t n3, int64_t p, int L,
                            int trans_a, int trans_b, int dtype, int gemm, void* stream);

/* Bytes of the fixed device scratch of w_product_noalloc. */
size_t w_product_noalloc_scratch_bytes(void);

/* ---- w-svd (Alg. 2, Thm 2.5) ------------------------------------------------
 * Truncated SVD of every coefficient slice of W(A), A (p, n1, n2), by one-sided
 * Jacobi.  Precision: the rotation parameters (cosine and sine, from the
 * tangent of the angle that zeroes the pair's inner product) are computed in
 * FP64 (to about one unit in the last place for WP_F64, to ~4e-15 relative for
 * WP_F32, whose rotations are applied in FP32); the column norms and the inner
 * product they come from are accumulated
 * in the data type (FP32 sums of FP32 products for WP_F32, FP64 for WP_F64);
 * the rotations are applied to the data in `dtype`.  The pair threshold is
 * |w_i.w_j| > sqrt(max(n1, n2)) * u * |w_i| |w_j| (u = 2^-24 for F32, 2^-53 for
 * F64); a slice has converged after a sweep with no rotation.  One factor is
 * formed from the converged columns; the other is recovered from the slice
 * (v_i = A^T u_i / sigma_i, or u_i = A v_i / sigma_i), accumulated in FP64,
 * and orthonormalised by Newton-Schulz steps in FP64 until it is orthonormal
 * to the rounding of `dtype` (at most 4 steps).  Outputs (wavelet-domain
 * factors, Thm 2.5):
 *   uhat (p, n1, k), shat (p, k) descending and >= 0, vhat (p, n2, k),
 *   ak (p, n1, n2) = W^{-1}(uhat_k diag(shat_k) vhat_k^T), or NULL to skip.
 * Numerical rank: a recovered column whose singular value is at or below
 *   max(n1, n2) * u * shat[slice][0] (the default cut of w_pinv) is returned
 *   zero, and so are the columns of zero singular values; they add nothing
 *   to ak.
 * Signs: in each column of uhat the entry of largest magnitude is positive
 * (lowest row wins ties); the matching vhat column is flipped with it.
 * info (p int32, device): sweeps used by slice k if it converged, minus the
 *   sweeps run if it did not (max_sweeps reached, or a non-finite value met).
 * orth_err (2 doubles, device, or NULL): max over slices of
 *   max|uhat^T uhat - I| and of max|vhat^T vhat - I|, evaluated in FP64 over
 *   the columns that are not zero.
 * 1 <= k <= min(n1, n2); max_sweeps >= 1 (<= 0 selects 30 for F64, 20 for F32);
 * n1, n2 <= 2048.  ws must hold w_svd_workspace(...) bytes.
 */
wp_status w_svd(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k,
                void* uhat, void* shat, void* vhat, void* ak, int max_sweeps,
                int32_t* info, double* orth_err, int dtype,
                void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for w_svd (0 on invalid arguments). */
size_t w_svd_workspace(int64_t n1, int64_t n2, int64_t p, int L, int k, int dtype);

/* w_svd, with two caller-owned HIP events (hipEvent_t, created by the caller
 * on the stream's device; either may be NULL) recorded on `stream` just before
 * and just after the Jacobi stage (the sweeps, the singular values and the
 * factor formed from the columns), so that hipEventElapsedTime times the
 * decomposition alone.  All other arguments, results and errors as for w_svd;
 * a failed hipEventRecord returns WP_ELAUNCH. */
wp_status w_svd_timed(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k,
                      void* uhat, void* shat, void* vhat, void* ak, int max_sweeps,
                      int32_t* info, double* orth_err, int dtype,
                      void* ws, size_t ws_bytes, void* stream,
                      void* jacobi_begin, void* jacobi_end);

/* ---- sp-w-svd (Sec. IV-B, computational analysis) ---------------------------
 * Sparse variant of w_svd: only the two coarsest coefficient blocks, s_L and
 * d_L (the leading nk = 2 p / 2^L slices of W(A)), are decomposed and
 * truncated; the finer details d_j, j < L, are dropped, so
 *   ak = W^{-1}(uhat_k diag(shat_k) vhat_k^T on the nk kept slices, 0 elsewhere).
 * Arguments, signs, info and orth_err are as for w_svd, except that uhat
 * (nk, n1, k), shat (nk, k), vhat (nk, n2, k) and info (nk) hold nk slices;
 * ak stays (p, n1, n2).  Requires L >= 1 (WP_EINVAL otherwise).
 */
wp_status w_svd_sparse(const void* a, int64_t n1, int64_t n2, int64_t p, int L, int k,
                       void* uhat, void* shat, void* vhat, void* ak, int max_sweeps,
                       int32_t* info, double* orth_err, int dtype,
                       void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for w_svd_sparse (0 on invalid arguments). */
size_t w_svd_sparse_workspace(int64_t n1, int64_t n2, int64_t p, int L, int k, int dtype);

/* ---- Moore-Penrose inverse (Def. 2.6, Thm 2.6; deblurring of Sec. IV-C) ------
 * out = A^+ = W^{-1}( V_c Sigma_c^+ U_c^T ) over the coefficient slices c of
 * W(A), A (p, n1, n2), out (p, n2, n1) (caller-allocated, device).  The
 * slice SVDs are the full-rank w-svd of w_svd; Sigma^+ inverts the singular
 * values above rtol * sigma_max of the slice and zeroes the rest.
 * rtol in [0, 1); 0 selects max(n1, n2) * machine epsilon of the data type.
 * sparse != 0 inverts only s_L and d_L (the first 2 p / 2^L coefficient
 * slices; needs L >= 1) and leaves the finer detail coefficients of A^+ zero
 * (the sp-w-product of Sec. IV-C).
 * info (device int32, one per inverted slice): Jacobi sweeps used by the
 *   slice, negative if it did not converge (see w_svd).
 * n1, n2 <= 2048.  ws must hold w_pinv_workspace(...) bytes.
 */
wp_status w_pinv(const void* a, void* out, int64_t n1, int64_t n2, int64_t p, int L,
                 int sparse, double rtol, int32_t* info, int dtype,
                 void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for w_pinv (0 on invalid arguments). */
size_t w_pinv_workspace(int64_t n1, int64_t n2, int64_t p, int L, int sparse, int dtype);

#ifdef __cplusplus
}
#endif

#endif /* WPROD_H */
