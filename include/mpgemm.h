/*
 * mpgemm.h -- C ABI of libmpgemm: double-double (DD), triple-double (TD) and
 * quad-double (QD) matrix multiplication on AMD Instinct MI355X (gfx950).
 *
 * The method is Kouya, "Acceleration of multiple precision matrix
 * multiplication based on multi-component floating-point arithmetic using
 * AVX2" (arXiv 2101.06584): numbers are unevaluated sums of P binary64
 * components (P = 2 DD, 3 TD, 4 QD; Sec. 2, component 0 most significant),
 * added and multiplied with the error-free-transformation algorithms of
 * Sec. 2.2-2.4 (Algorithms 1, 2, 4, 5, 6; TD addition = QD addition with zero
 * fourth components), and the product is eqn (1) of Sec. 3 extended to the
 * BLAS form C = alpha op(A) op(B) + beta C of the Rgemm routine the paper
 * benchmarks against.
 *
 * Storage (Sec. 2.5, Fig. 1: one array per component): every matrix is P
 * column-major "component planes" of device memory.  Element (i, j) of
 * component p of X is X[p * x_plane_stride + i + j * ldx].  Scalars alpha and
 * beta are host arrays of P doubles.  All matrix pointers are device pointers
 * owned by the caller; the library never frees or retains them.
 *
 * Semantics (as BLAS xGEMM):
 *   op(X) = X for 'N'/'n', X^T for 'T'/'t'/'C'/'c' (real data: 'C' == 'T').
 *   op(A) is m x k, op(B) is k x n, C is m x n.
 *   Quick return (nothing launched) when m == 0, n == 0, or when alpha == 0
 *   or k == 0 and beta == 1 exactly.  alpha == 0 or k == 0 otherwise gives
 *   C = beta C (C = 0 when beta == 0).  When beta == 0, C is never read.
 *   "== 0" means every component is zero; "== 1" means (1, 0, ..., 0).
 *   C must not overlap A or B.
 *
 * Errors: 0 on success.  A negative value -i reports that the i-th argument
 * (1-based, in signature order) is invalid; checks run on the host before
 * any GPU work, in argument order, and never print or abort.  Positive
 * values are runtime failures (MPGEMM_ERR_*), see mpgemm_strerror().
 * Launches are asynchronous on `stream`; faults inside a kernel surface at
 * the caller's next synchronisation.  No C++ exception crosses this ABI.
 */
#ifndef MPGEMM_H
#define MPGEMM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Positive error codes. */
#define MPGEMM_ERR_HIP 1          /* a HIP runtime call or launch failed        */
#define MPGEMM_ERR_WORKSPACE 2    /* split form: workspace missing or too small */
#define MPGEMM_ERR_UNSUPPORTED 3  /* shape or option outside what a form does   */
#define MPGEMM_ERR_GRAPH 4        /* hipGraph capture / instantiation failed    */
#define MPGEMM_ERR_ALIAS 5        /* C overlaps A or B                          */
#define MPGEMM_ERR_NOMEM 6        /* host or device allocation failed           */
#define MPGEMM_ERR_SCRATCH 7      /* mpgemm_ex_noalloc: the call needs more than
                                     MPGEMM_STATIC_SCRATCH_BYTES of scratch    */

/* Precision ids (the number of binary64 components). */
#define MPGEMM_DD 2
#define MPGEMM_TD 3
#define MPGEMM_QD 4

/* Forms. */
#define MPGEMM_FORM_PLAIN 0     /* FP64-VALU EFT kernel; bitwise equal to the
                                   canonical ascending-k evaluation         */
#define MPGEMM_FORM_SPLIT_I8 1  /* operands cut into signed 7-bit INT8 digits,
                                   exact INT8 MFMA digit products, exact
                                   recombination into P components          */
#define MPGEMM_FORM_AUTO 2      /* the library's choice.  With opts.slices
                                   = 0: plain.  With opts.slices = s > 0
                                   (the caller's digit count, e.g. from
                                   mpgemm_tune_slices): the residue form
                                   (MPGEMM_FORM_SPLIT_CRT) for m, n, k >= 128
                                   (DD), 96 (TD) or 64 (QD) when the
                                   workspace (256-byte aligned) holds it and
                                   it applies, else for m, n, k >= 256 the
                                   split form when the workspace holds that,
                                   else plain; never a workspace error.
                                   The split forms' error bound depends on
                                   the spread of magnitudes within each row
                                   of op(A) and column of op(B) (see
                                   opts.slices), which the library does not
                                   inspect; choosing s is the caller's
                                   accuracy decision                      */
#define MPGEMM_FORM_STRASSEN 4  /* Strassen's method (Sec. 3, Fig. 5): opts.levels
                                   levels of the seven-product recursion over
                                   plain-form block products               */
#define MPGEMM_FORM_SPLIT_CRT 5 /* residue form of the split product: the
                                   same digits, their integer product over
                                   the full square of digit pairs from one
                                   INT8 product per coprime modulus        */

/* TD operation variants (Sec. 2.3).  The defaults are TDaddq (the QD
 * addition on zero fourth components) and the "fast" triple-word product
 * (Algorithm 4). */
#define MPGEMM_TD_ADD_ACCURATE 1  /* Algorithm 3: Merge by decreasing magnitude,
                                     VecSum of the six terms, VSEB(3)        */
#define MPGEMM_TD_MULQ 2          /* TDmulq: the QD product (Algorithm 6) on
                                     zero fourth components, fourth output
                                     dropped                                 */

/* Options for the _ex entry points.  Zero-initialise and set what you need. */
typedef struct mpgemm_opts {
    int form;               /* MPGEMM_FORM_*                                   */
    int slices;             /* split forms: digits per operand entry s (1..40);
                               0 = the precision's default (DD 16, TD 23, QD 31),
                               enough for inputs of similar magnitude within a
                               row of op(A) / column of op(B).  The dropped
                               digits of entry a_il weigh up to 2^(E_i - 7 s - 1)
                               whatever |a_il| is, so entries far below their
                               row's largest need more digits to stay within
                               8 k u (|A||B|)_ij; mpgemm_tune_slices picks s
                               for given operands.  MPGEMM_FORM_AUTO takes a
                               split form only when s is given             */
    int tile;               /* kernel configuration id; -1 or 0.. = tuned/fixed */
    int variant;            /* TD only, plain form: MPGEMM_TD_* bits selecting
                               the other TD operations of Sec. 2.3 (runs TD
                               tile configuration 0); 0 = the defaults      */
    void* workspace;        /* split / Strassen form: device scratch owned by
                               the caller, 256-byte aligned; a call uses it
                               until its kernels end on `stream`, so calls
                               that may overlap (other streams) need their
                               own workspaces                               */
    size_t workspace_bytes; /* its size; see mpgemm_workspace_bytes()          */
    int levels;             /* Strassen form: recursion levels L (1..5; 0 = 1);
                               m, n, k must be multiples of 2^L            */
} mpgemm_opts;

/*
 * C = alpha op(A) op(B) + beta C in DD (P = 2), TD (P = 3) and QD (P = 4),
 * plain form.  Arguments, in order (error code -i names argument i):
 *   1 transa, 2 transb: 'N','n','T','t','C','c'
 *   3 m, 4 n, 5 k: >= 0
 *   6 alpha: host pointer to P doubles (non-NULL)
 *   7 A: device pointer (may be NULL only if A is not read: m, n or k == 0 or
 *        alpha == 0); 8 lda >= max(1, rows of A) (m if 'N', else k);
 *   9 a_plane_stride >= lda * (columns of A), so planes never overlap
 *  10 B, 11 ldb >= max(1, rows of B) (k if 'N', else n), 12 b_plane_stride
 *  13 beta: host pointer to P doubles (non-NULL)
 *  14 C: device pointer (non-NULL when m, n > 0), 15 ldc >= max(1, m),
 *  16 c_plane_stride >= ldc * n
 *  17 stream: HIP stream the kernels are queued on (0 = null stream)
 * The result is bitwise identical to evaluating, for every entry, one
 * running sum acc = ADD(acc, MUL(op(A)_il, op(B)_lj)) for l = 0..k-1 and then
 * ADD(MUL(alpha, acc), MUL(beta, c)) (MUL(alpha, acc) when beta == 0).
 */
int mpgemm_dd(char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
              const double* A, int64_t lda, int64_t a_plane_stride, const double* B, int64_t ldb,
              int64_t b_plane_stride, const double* beta, double* C, int64_t ldc,
              int64_t c_plane_stride, hipStream_t stream);
int mpgemm_td(char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
              const double* A, int64_t lda, int64_t a_plane_stride, const double* B, int64_t ldb,
              int64_t b_plane_stride, const double* beta, double* C, int64_t ldc,
              int64_t c_plane_stride, hipStream_t stream);
int mpgemm_qd(char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
              const double* A, int64_t lda, int64_t a_plane_stride, const double* B, int64_t ldb,
              int64_t b_plane_stride, const double* beta, double* C, int64_t ldc,
              int64_t c_plane_stride, hipStream_t stream);

/*
 * As above with options (argument 18, non-NULL; -18 if malformed).
 * form = MPGEMM_FORM_SPLIT_I8: every row i of op(A) is scaled by 2^-E_i and
 * every column j of op(B) by 2^-F_j (powers of two from the largest leading
 * component), cut into s signed digits of 7 bits in [-64, 64]; the digit
 * products of pairs (p, q) with p + q <= s + 1 are summed exactly in 32-bit
 * integers on the INT8 matrix cores, one anti-diagonal p + q = d at a time;
 * X_ij = sum_d S_d 128^(s+1-d) is formed exactly and X_ij 2^(E_i + F_j -
 * 7 (s+1)) rounded once into P components (repeated round to nearest, ties
 * to even, of the exact remainder), then the plain epilogue applied.  Not
 * the canonical evaluation order, so the result differs in the last bits;
 * with enough digits its error stays within 8 (k+2) u (|alpha||A||B| +
 * |beta||C|) componentwise.  Needs opts->workspace of at least
 * mpgemm_workspace_bytes() bytes (device memory the caller owns; no
 * allocation on this path).  Supported for k * s <= 2^19 (exact 32-bit
 * accumulation); larger k returns MPGEMM_ERR_UNSUPPORTED.  The split forms
 * (this one and MPGEMM_FORM_SPLIT_CRT) need finite operands: digits of an
 * Inf or NaN do not exist, so with one in op(A) or op(B) the result is
 * unspecified (finite garbage in the rows and columns it scales; no memory
 * outside the buffers is touched).  The plain form follows IEEE arithmetic.
 * form = MPGEMM_FORM_STRASSEN: C = alpha P + beta C (the plain epilogue) with
 * P from opts->levels levels of Strassen's method: op(A), op(B) and P cut into
 * 2 x 2 blocks, P from the seven block products
 *   M1 = (A11 + A22)(B11 + B22), M2 = (A21 + A22) B11, M3 = A11 (B12 - B22),
 *   M4 = A22 (B21 - B11), M5 = (A11 + A12) B22, M6 = (A21 - A11)(B11 + B12),
 *   M7 = (A12 - A22)(B21 + B22); P11 = M1 + M4 - M5 + M7, P12 = M3 + M5,
 *   P21 = M2 + M4, P22 = M1 - M2 + M3 + M6
 * (sums left to right, x - y as x + (-y) with exact negation), recursively;
 * the bottom blocks are plain-form products.  Deterministic; its error bound
 * is normwise (Strassen's), not componentwise.  m, n, k not multiples of
 * 2^levels return MPGEMM_ERR_UNSUPPORTED; needs opts->workspace (256-byte
 * aligned) of mpgemm_workspace_bytes(prec, MPGEMM_FORM_STRASSEN, m, n, k,
 * levels, -1) bytes.
 * form = MPGEMM_FORM_SPLIT_CRT: the split form's scaling and s digits per
 * entry define integers A'_il = sum_p d_p 128^(s-p) and B'_lj; the exact
 * C'_ij = sum_l A'_il B'_lj is reconstructed (Chinese remainder theorem) from
 * its residues modulo the first N of 49 pairwise coprime moduli <= 256, one
 * exact INT8 matrix-core product per modulus, N the smallest count whose
 * product M exceeds 2 k (64 (128^s - 1) / 127)^2; then C'_ij 2^(E_i + F_j -
 * 14 s) is rounded to P components by repeated round to nearest (ties to
 * even) of the exact remainder and the plain epilogue applied.  N grows with
 * 14 s + log2 k (DD, s = 16: at most 32 moduli; TD, s = 23: 48 for k <= 2^13,
 * 49 above).  QD with 25 <= s <= 32 digits (its default s = 31 included), where
 * 49 moduli do not suffice, cuts each digit integer into a high half of
 * ceil(s/2) digits and a low half, A' = A_h 128^floor(s/2) + A_l, and forms C' =
 * hh 128^(2 floor(s/2)) + (ss - hh - ll) 128^floor(s/2) + ll from the three
 * half-size products hh = A_h B_h, ll = A_l B_l, ss = (A_h + A_l)(B_h + B_l),
 * each from N <= 33 moduli: the same integer, so the same result.
 * MPGEMM_ERR_UNSUPPORTED otherwise (s > 24 for DD and TD, s > 32 for QD,
 * k > 131071, or s = 24 with k > 114, where 49 moduli do not suffice: the
 * count is taken from logarithms with a margin of 0.01 bit).  Deterministic; the exactly rounded product of the truncated
 * operands.  Workspace as for the split form, sized by
 * mpgemm_workspace_bytes(prec, MPGEMM_FORM_SPLIT_CRT, m, n, k, slices, tile).
 * opts->variant (TD, plain form only; MPGEMM_ERR_UNSUPPORTED for another
 * precision or the split forms, -18 outside 0..3): the same canonical
 * evaluation with the accurate TD addition (MPGEMM_TD_ADD_ACCURATE) and / or
 * TDmulq (MPGEMM_TD_MULQ) in place of TDaddq and Algorithm 4, everywhere
 * including the alpha/beta epilogue; FORM_AUTO then means plain.
 */
int mpgemm_dd_ex(char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
                 const double* A, int64_t lda, int64_t a_plane_stride, const double* B, int64_t ldb,
                 int64_t b_plane_stride, const double* beta, double* C, int64_t ldc,
                 int64_t c_plane_stride, hipStream_t stream, const mpgemm_opts* opts);
int mpgemm_td_ex(char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
                 const double* A, int64_t lda, int64_t a_plane_stride, const double* B, int64_t ldb,
                 int64_t b_plane_stride, const double* beta, double* C, int64_t ldc,
                 int64_t c_plane_stride, hipStream_t stream, const mpgemm_opts* opts);
int mpgemm_qd_ex(char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
                 const double* A, int64_t lda, int64_t a_plane_stride, const double* B, int64_t ldb,
                 int64_t b_plane_stride, const double* beta, double* C, int64_t ldc,
                 int64_t c_plane_stride, hipStream_t stream, const mpgemm_opts* opts);

/*
 * For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the same call as
 * mpgemm_{dd,td,qd}_ex for precision `prec` (argument 1: 2, 3 or 4; the
 * other arguments follow as arguments 2..19, so an invalid argument i of
 * the _ex entry point is reported as -(i + 1)), except that the split,
 * residue and Strassen forms take their scratch from a buffer of
 * MPGEMM_STATIC_SCRATCH_BYTES bytes that the library holds in static device
 * memory, one per GPU, from the first call on that GPU until the process
 * ends.  opts->workspace must be NULL and opts->workspace_bytes 0 (-19
 * otherwise).  The call allocates nothing (no hipMalloc, no hipFree); the
 * first call on a device looks up the buffer's device address once, with
 * that device current.  A form whose workspace (mpgemm_workspace_bytes)
 * exceeds the buffer returns MPGEMM_ERR_SCRATCH before any GPU work;
 * MPGEMM_FORM_AUTO never does: it takes the residue or split form only when
 * it fits, else plain.  Results are bitwise those of the _ex call with the
 * same opts and a workspace of its own.  Every call on a GPU shares that
 * GPU's buffer: calls that may overlap (queued on different streams, or
 * from several threads without ordering) race and give wrong results; calls
 * ordered on one stream are safe.  The kernels write every scratch byte they
 * read, so nothing carries over from one call to the next.
 */
#define MPGEMM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int mpgemm_ex_noalloc(int prec, char transa, char transb, int64_t m, int64_t n, int64_t k,
                      const double* alpha, const double* A, int64_t lda, int64_t a_plane_stride,
                      const double* B, int64_t ldb, int64_t b_plane_stride, const double* beta,
                      double* C, int64_t ldc, int64_t c_plane_stride, hipStream_t stream,
                      const mpgemm_opts* opts);

/* Residue form: the number of INT8 products a call runs for inner dimension
 * k and s digits per entry (slices 0 = the default of precision prec): the
 * modulus count N, or 3 N with two levels (QD, s > 24); 0 when the form does
 * not apply (too many digits, or k outside 1..131071); -1 for an invalid
 * precision. */
int mpgemm_crt_moduli(int prec, int64_t k, int slices);

/* Workspace bytes the split forms (MPGEMM_FORM_SPLIT_I8, _AUTO, _SPLIT_CRT)
 * need for this shape (0 for the plain form; for the residue form also 0 when
 * no modulus count suffices; for _AUTO the larger of the two split forms'
 * needs, so that either fits; slices 0 = default; tile -1 = the one the
 * library would pick); for
 * MPGEMM_FORM_STRASSEN, `slices` is the number of levels L (0 = 1) and the
 * result is 8 P (m n + sum over l = 1..L of 7^l (m k + k n + m n) / 4^l)
 * bytes (the product and, per level, operands and results of its 7^l
 * nodes).  Returns 0 for invalid arguments. */
size_t mpgemm_workspace_bytes(int prec, int form, int64_t m, int64_t n, int64_t k, int slices,
                              int tile);

/*
 * Element-wise vector operations of Sec. 2.5 (componentwise sums and
 * products of DD/TD/QD vectors): r_i = x_i + y_i (add) or
 * x_i * y_i (mul), i < n, with each vector stored as P planes of n doubles at
 * plane strides sx, sy, sr (device pointers; r may equal x or y).
 * Arguments: 1 n >= 0, 2 x, 3 sx >= n, 4 y, 5 sy >= n, 6 r, 7 sr >= n, 8 stream.
 */
int mp_vec_dd_add(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* r,
                  int64_t sr, hipStream_t stream);
int mp_vec_dd_mul(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* r,
                  int64_t sr, hipStream_t stream);
int mp_vec_td_add(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* r,
                  int64_t sr, hipStream_t stream);
int mp_vec_td_mul(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* r,
                  int64_t sr, hipStream_t stream);
int mp_vec_qd_add(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* r,
                  int64_t sr, hipStream_t stream);
int mp_vec_qd_mul(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* r,
                  int64_t sr, hipStream_t stream);
/* The other TD operations of Sec. 2.3, element-wise, same arguments:
 * the accurate addition (Algorithm 3) and TDmulq (see MPGEMM_TD_*). */
int mp_vec_td_add_acc(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy,
                      double* r, int64_t sr, hipStream_t stream);
int mp_vec_td_mulq(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* r,
                   int64_t sr, hipStream_t stream);

/*
 * BLAS-1/2 in DD / TD / QD (the vector kernels that accompany the paper's
 * Strassen code, Sec. 4).  Vectors are P planes of doubles at the given plane
 * strides (device pointers); scalars are host arrays of P doubles.  Error
 * codes: -(argument position) as for the GEMM entry points.
 *
 * axpy: y_i = ADD(MUL(alpha, x_i), y_i), i < n.  Arguments: 1 n >= 0,
 *   2 alpha, 3 x, 4 sx >= n, 5 y (may equal x), 6 sy >= n, 7 stream.
 */
int mp_axpy_dd(int64_t n, const double* alpha, const double* x, int64_t sx, double* y, int64_t sy,
               hipStream_t stream);
int mp_axpy_td(int64_t n, const double* alpha, const double* x, int64_t sx, double* y, int64_t sy,
               hipStream_t stream);
int mp_axpy_qd(int64_t n, const double* alpha, const double* x, int64_t sx, double* y, int64_t sy,
               hipStream_t stream);

/*
 * dot: result = sum_i x_i y_i in a fixed order: the products in blocks of 64
 * consecutive terms, each block summed from zero in ascending order
 * (acc = ADD(acc, MUL(x_i, y_i))), then the block sums 64 at a time the same
 * way, until one value is left (for n <= 64 the sequential chain).  The
 * P-component result is written to device memory at `result` (asynchronously,
 * on the stream).  Partial sums use the caller's workspace of
 * mp_dot_workspace_bytes(prec, n) bytes (0 when n <= 64; NULL allowed then).
 * Arguments: 1 n >= 0, 2 x, 3 sx >= n, 4 y, 5 sy >= n, 6 result, 7 workspace,
 * 8 workspace_bytes (MPGEMM_ERR_WORKSPACE if short), 9 stream.
 */
size_t mp_dot_workspace_bytes(int prec, int64_t n);
int mp_dot_dd(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* result,
              void* workspace, size_t workspace_bytes, hipStream_t stream);
int mp_dot_td(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* result,
              void* workspace, size_t workspace_bytes, hipStream_t stream);
int mp_dot_qd(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* result,
              void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * gemv: y = alpha op(A) x + beta y for A stored m x n (column-major, planes at
 * a_plane_stride), y of length rows(op(A)) and x of length cols(op(A)); each
 * entry bitwise as the plain GEMM with one column (canonical ascending chain,
 * same epilogue, C = y never read when beta == 0, quick return when alpha or
 * the inner length is 0 and beta == 1).  Arguments: 1 trans, 2 m >= 0,
 * 3 n >= 0, 4 alpha, 5 A, 6 lda >= max(1, m), 7 a_plane_stride >= lda n, 8 x,
 * 9 sx >= cols(op(A)), 10 beta, 11 y, 12 sy >= rows(op(A)), 13 stream;
 * MPGEMM_ERR_ALIAS if y overlaps A or x.
 */
int mp_gemv_dd(char trans, int64_t m, int64_t n, const double* alpha, const double* A, int64_t lda,
               int64_t a_plane_stride, const double* x, int64_t sx, const double* beta, double* y,
               int64_t sy, hipStream_t stream);
int mp_gemv_td(char trans, int64_t m, int64_t n, const double* alpha, const double* A, int64_t lda,
               int64_t a_plane_stride, const double* x, int64_t sx, const double* beta, double* y,
               int64_t sy, hipStream_t stream);
int mp_gemv_qd(char trans, int64_t m, int64_t n, const double* alpha, const double* A, int64_t lda,
               int64_t a_plane_stride, const double* x, int64_t sx, const double* beta, double* y,
               int64_t sy, hipStream_t stream);

/*
 * Batched GEMMs of uneven shapes (an addition to the paper's single GEMM).
 * Plain form: one persistent launch, the same per-entry results as one
 * mpgemm_*() call per problem.  Residue form (opts->form
 * MPGEMM_FORM_SPLIT_CRT, or _AUTO with opts->slices > 0 for the problems the
 * single call's AUTO rule would give it by size): each of its four stages
 * (scale exponents, residues, one INT8 product per modulus, exact
 * reconstruction) is one launch over all residue problems, with every
 * problem's result bitwise that of a single residue-form call with the same
 * s.  A problem is the argument list of mpgemm_dd() as a struct; alpha/beta
 * use the first P entries.  Problems must not write overlapping C regions.
 */
typedef struct mpgemm_problem {
    char transa, transb;
    int64_t m, n, k;
    double alpha[4];
    double beta[4];
    const double* A;
    int64_t lda, a_plane_stride;
    const double* B;
    int64_t ldb, b_plane_stride;
    double* C;
    int64_t ldc, c_plane_stride;
} mpgemm_problem;

typedef struct mpgemm_batch_plan mpgemm_batch_plan;  /* opaque */

/*
 * Build a plan: validates every problem (error -(1000 + index) for an
 * invalid problem; its first bad field is not reported separately), orders
 * tiles largest-k first, copies the descriptors to device memory owned by
 * the plan, and captures every launch of a run in a hipGraph.  Arguments:
 * 1 prec (2, 3, 4), 2 count >= 0, 3 problems (host array of count), 4 opts
 * (may be NULL = plain; -4 if its fields are out of range; opts->tile selects
 * the plain part's tile shape; form MPGEMM_FORM_PLAIN, _AUTO or _SPLIT_CRT,
 * else MPGEMM_ERR_UNSUPPORTED, as for variant != 0), 5 stream used for the
 * uploads, 6 out (receives the plan).
 * Residue form: opts->slices = s digits (0 = the precision's default for
 * _SPLIT_CRT); every problem with m, n, k > 0 and alpha != 0 takes it, and
 * the plan returns MPGEMM_ERR_UNSUPPORTED when one has no residue product
 * (k beyond its range); the rest (a zero alpha or dimension) run in the
 * plain part.  Every residue problem uses the moduli, and the levels (two
 * for QD with s > 24, as in the single call), that the largest k among them
 * needs (the reconstruction is exact, so extra moduli change no bit).  The plan owns the residue workspace
 * (problems padded to 128 x 128 product tiles, grouped into chunks that
 * run one after another, each within opts->workspace_bytes if nonzero, else
 * 8 GiB; opts->workspace itself is not used; mpgemm_batch_plan_residue_info
 * reports the chunks and bytes).
 * The plan binds the device addresses in `problems`; their contents may
 * change between runs.
 */
int mpgemm_batch_plan_create(int prec, int64_t count, const mpgemm_problem* problems,
                             const mpgemm_opts* opts, hipStream_t stream,
                             mpgemm_batch_plan** out);
/* Replay the captured graph on `stream`.  A plan holds one device tile
 * counter that each run (graph replay or direct launch) resets and then
 * consumes, and one residue workspace that each run overwrites, so the runs
 * of one plan must not overlap: queue them on one stream, or order the
 * streams (events).  Overlapping runs of the same plan skip or repeat tiles
 * or mix their residues and give wrong results; different plans are
 * independent. */
int mpgemm_batch_plan_run(mpgemm_batch_plan* plan, hipStream_t stream);
/* Same work as a direct launch (no graph) on `stream`; ordered like runs. */
int mpgemm_batch_plan_launch(mpgemm_batch_plan* plan, hipStream_t stream);
/* Plain part: total tiles, the persistent grid and its tile shape (for
 * reporting). */
int mpgemm_batch_plan_info(const mpgemm_batch_plan* plan, int64_t* tiles, int* grid, int* tile_cfg);
/* Residue part: problems, INT8 products per problem (as mpgemm_crt_moduli:
 * N, or 3 N with two levels), chunks and the workspace bytes the plan holds
 * for them (any pointer may be NULL). */
int mpgemm_batch_plan_residue_info(const mpgemm_batch_plan* plan, int64_t* problems, int* moduli, int* chunks,
                                   size_t* workspace_bytes);
/* Free the plan's device memory and graph (after its last run completed). */
int mpgemm_batch_plan_destroy(mpgemm_batch_plan* plan);

/*
 * Grouped calls (the batched form in one call): all `count` problems of one
 * precision computed by a batched plan replayed from a hipGraph, each problem
 * bitwise as one single call in its form (plain, or residue with the same s).  The first call with a given
 * problem array (every field compared, device addresses included) builds a
 * plan as mpgemm_batch_plan_create does (device allocations, graph capture;
 * not to be called under stream capture); later calls with an equal array
 * replay it.  The library keeps the 8 most recently used plans, each with
 * its device memory (a residue plan's workspace up to the default 8 GiB
 * chunk bound; opts->workspace_bytes is not used here); dropping one
 * synchronises the device first; mpgemm_finalize releases them.  Calls with
 * equal arrays reuse one plan, so they follow the plan rule: queue them on
 * one stream or order the streams.  Arguments: 1 count >= 0, 2 problems
 * (host array; -(1000 + index) for an invalid problem), 3 opts (may be NULL;
 * form MPGEMM_FORM_PLAIN, _AUTO or _SPLIT_CRT with opts->slices as for
 * mpgemm_batch_plan_create, variant 0, opts->tile selects the plain tile
 * shape, -1 = tuned; form, slices and tile are part of the plan's key),
 * 4 stream.
 */
int mpgemm_dd_grouped(int64_t count, const mpgemm_problem* problems, const mpgemm_opts* opts,
                      hipStream_t stream);
int mpgemm_td_grouped(int64_t count, const mpgemm_problem* problems, const mpgemm_opts* opts,
                      hipStream_t stream);
int mpgemm_qd_grouped(int64_t count, const mpgemm_problem* problems, const mpgemm_opts* opts,
                      hipStream_t stream);

/*
 * Autotuner: times every kernel configuration of a form (MPGEMM_FORM_PLAIN,
 * _SPLIT_I8 or _SPLIT_CRT) on a problem of the given shape (synthetic operands allocated by the tuner; not a hot path) and
 * records the fastest for that precision / form / shape bucket (log2 of m, n,
 * k).  Later calls with tile = -1 (or the non-_ex entry points) use it.
 * Writes the chosen configuration id to *best (may be NULL).
 */
int mpgemm_autotune(int prec, int form, int64_t m, int64_t n, int64_t k, int slices,
                    hipStream_t stream, int* best);
/* Batched form: times every tile configuration on these problems (plans are
 * built and destroyed by the call; the problems' C buffers are overwritten)
 * and records the fastest under form id 3 for the problems' mean shape.
 * Arguments as mpgemm_batch_plan_create; *best (may be NULL) gets the id. */
int mpgemm_batch_autotune(int prec, int64_t count, const mpgemm_problem* problems,
                          hipStream_t stream, int* best);
/* Record a configuration for a precision / form (0 plain, 1 split, 3 batched,
 * 5 residue split) / shape bucket directly (e.g. from a table produced elsewhere). */
int mpgemm_autotune_set(int prec, int form, int64_t m, int64_t n, int64_t k, int tile);
/* Persist / restore the tuning table as a small text file: a header line
 * naming the format and the architecture (gfx950), then one entry per line:
 * prec form log2m log2n log2k tile signature, the signature (hex) that of
 * the configuration list of that precision and form when the entry was
 * made.  Loading adds the entries whose signature matches the library's
 * current configurations and skips the others (0); a file of another format
 * or architecture returns MPGEMM_ERR_UNSUPPORTED, an unreadable one
 * MPGEMM_ERR_HIP.  The library loads a table by itself at the first use of
 * the tuning choices: the file MPGEMM_AUTOTUNE_CACHE names, else
 * tuned_gfx950.txt beside libmpgemm.so; none when MPGEMM_NO_TUNED_TABLE is
 * set.  mpgemm_autotune_load adds a file's entries on top. */
int mpgemm_autotune_save(const char* path);
int mpgemm_autotune_load(const char* path);
/* Number of configurations a form offers for a precision. */
int mpgemm_num_configs(int prec, int form);

/*
 * Pick the slice count of the split form by an accuracy rule: on a block of
 * up to 64 rows of op(A) it compares the split result for s = smin, smin+1,
 * ... against the plain (canonical) result and returns the smallest s whose
 * largest difference, relative to k u (|A||B|)_ij, is at most `target`
 * (u = 2^-104 DD, 2^-150 TD, 2^-200 QD).  Scratch is allocated by the call.
 * Same argument conventions as mpgemm_dd() for the matrices.
 */
int mpgemm_tune_slices(int prec, char transa, char transb, int64_t m, int64_t n, int64_t k,
                       const double* A, int64_t lda, int64_t a_plane_stride, const double* B,
                       int64_t ldb, int64_t b_plane_stride, double target, int smin, int smax,
                       hipStream_t stream, int* s_out, double* ratio_out);

/*
 * Stages of the split form, exposed so each can be checked on its own.
 * They operate on a workspace laid out by the library for (prec, m, n, k, s,
 * tile); offsets (bytes) and padded sizes are reported by
 * mpgemm_split_layout.  Digit planes are int8 [s][Kp/64][Mp][64] (op(A)
 * rows) and [s][Kp/64][Np][64] (op(B) columns): digit p of entry (r, l) is at
 * ((p-1) (Kp/64) + l/64) Rp 64 + r 64 + l % 64; exponents are int32 [Mp], [Np];
 * anti-diagonal sums are int32 [s][Np][Mp] (d = 2..s+1, column-major).
 */
int mpgemm_split_layout(int prec, int64_t m, int64_t n, int64_t k, int slices, int tile,
                        size_t* off_E, size_t* off_F, size_t* off_DA, size_t* off_DB,
                        size_t* off_S, int64_t* Mp, int64_t* Np, int64_t* Kp);
/* Run the stages up to and including `last` (1 = scale exponents, 2 = digit
 * slicing, 3 = anti-diagonal sums, 4 = recombination and epilogue = the full
 * product) with the same arguments as mpgemm_*_ex. */
int mpgemm_split_stages(int prec, int last, char transa, char transb, int64_t m, int64_t n,
                        int64_t k, const double* alpha, const double* A, int64_t lda,
                        int64_t a_plane_stride, const double* B, int64_t ldb,
                        int64_t b_plane_stride, const double* beta, double* C, int64_t ldc,
                        int64_t c_plane_stride, hipStream_t stream, const mpgemm_opts* opts);

/*
 * Measure a throughput peak of the GPU that `stream` runs on, as the figure
 * the GEMM kernels are compared with (not a hot-path call):
 *   which = 0: FP64 FMA, in flops/s (2 per FMA);
 *   which = 1: FP64 add, in operations/s;
 *   which = 2: FP64 multiply, in operations/s;
 *   which = 3: INT8 matrix cores (v_mfma_i32_32x32x32_i8), in operations/s
 *              (2 per multiply-add);
 *   which = 4: HBM, a streaming copy of 1 GiB with the element-wise kernels'
 *              access pattern, in bytes/s (read + written).
 * Each thread (FP64) or wave (MFMA) runs independent chains over 4096
 * workgroups of 256 threads for a few milliseconds; *rate is the best of three
 * timed launches after one warm-up.  Allocates and frees a scratch buffer
 * (8 MiB; 2 GiB for the copy); synchronises on the stream.  Returns -1 for a
 * bad `which`, -3 for a NULL `rate`, MPGEMM_ERR_NOMEM or MPGEMM_ERR_HIP on
 * failure.
 */
int mpgemm_probe_peak(int which, hipStream_t stream, double* rate);

/* Message for an error code; never NULL. */
const char* mpgemm_strerror(int code);
/* Library version string. */
const char* mpgemm_version(void);
/* Release library-owned state: the tuning table (looked for again at the
 * next use) and the grouped calls' plans (after a device synchronisation).
 * Plans made with mpgemm_batch_plan_create are freed separately. */
void mpgemm_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* MPGEMM_H */
