// internal.hpp -- host-side declarations shared by the kernel translation
// units and the C-ABI layer (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpgemm.h"

namespace mpg {

// One GEMM C = alpha op(A) op(B) + beta C on component planes (column-major
// planes, plane strides sa/sb/sc in elements).
struct GemmArgs {
    int64_t m, n, k;
    const double* A;
    int64_t lda, sa;
    const double* B;
    int64_t ldb, sb;
    double* C;
    int64_t ldc, sc;
    int ta, tb;            // 1 = transposed
    double alpha[4];
    double beta[4];
};

// Plain (FP64-VALU EFT) tile configurations.
struct PlainConfig {
    int tx, ty, tm, tn, bk;   // threads x/y, per-thread rows/cols, k tile
};

constexpr int kPlainConfigs = 4;
PlainConfig plain_config(int P, int id);
int plain_default_config(int P, int64_t m, int64_t n, int64_t k);

// Launchers return a hipError_t value (0 on success).
int launch_plain(int P, int cfg, const GemmArgs& g, hipStream_t st);
// `batch` equal-shape products, problem z at A + z zA, B + z zB, C + z zC
int launch_plain_strided(int P, int cfg, const GemmArgs& g, int64_t batch, int64_t zA, int64_t zB,
                         int64_t zC, hipStream_t st);
int launch_scale(int P, const GemmArgs& g, hipStream_t st);   // alpha == 0 or k == 0
int launch_plain_td_variant(int variant, const GemmArgs& g, hipStream_t st);

// Strassen's method over the plain form (strassen.hip).
size_t strassen_workspace_bytes(int P, int levels, int64_t m, int64_t n, int64_t k);
int launch_strassen(int P, int levels, const GemmArgs& g, void* ws, hipStream_t st,
                    int (*pick)(int, int64_t, int64_t, int64_t));
int launch_scale_td_variant(int variant, const GemmArgs& g, hipStream_t st);
int launch_vec(int P, int op, int64_t n, const double* x, int64_t sx, const double* y,
               int64_t sy, double* r, int64_t sr, hipStream_t st);

// Batched persistent form.  Device descriptor layout is private to the
// kernel file; these helpers size and fill it.
struct BatchProblemHost {
    GemmArgs g;
};
size_t batch_desc_bytes(int64_t count);
// Fills a host staging buffer with descriptors (tile prefix sums included);
// returns total tile count.  order[] gives the processing order.
int64_t batch_build_desc(int P, int cfg, int64_t count, const GemmArgs* probs, const int64_t* order,
                         void* host_buf);
int launch_batch(int P, int cfg, int64_t count, int64_t total_tiles, const void* dev_desc,
                 unsigned* dev_counter, int grid, hipStream_t st);
int batch_max_grid(int P, int cfg);

// Split (sliced INT8, MFMA) form.
struct SplitConfig {
    int bm, bn;                 // output tile per workgroup
    int g;                      // diagonals accumulated at once
};
constexpr int kSplitConfigs = 4;
SplitConfig split_config(int id);
size_t split_workspace_bytes(int P, int64_t m, int64_t n, int64_t k, int s, int cfg);
int launch_split(int P, int s, int cfg, const GemmArgs& g, void* ws, size_t ws_bytes,
                 hipStream_t st);
// Stage entry points for testing the split pipeline piece by piece.
int split_layout(int P, int64_t m, int64_t n, int64_t k, int s, int cfg, size_t* offE, size_t* offF,
                 size_t* offDA, size_t* offDB, size_t* offS, int64_t* Mp, int64_t* Np, int64_t* Kp);

// Scale exponents of the split forms (stage 1 above) for op(A)'s rows and
// op(B)'s columns: row r of a matrix whose element (r, l) sits at
// X[r rs + l ls]; E[r] = 0 for count <= r < padded (m, Mp for op(A) into E;
// n, Np for op(B) into F); mx: scratch of Mp + Np 64-bit words (device).
int launch_row_exponents(const double* A, int64_t a_rs, int64_t a_ls, int64_t m, int64_t Mp,
                         const double* B, int64_t b_rs, int64_t b_ls, int64_t n, int64_t Np,
                         int64_t k, int32_t* E, int32_t* F, uint64_t* mx, hipStream_t st);

// Residue (CRT) form of the split product (crt_gemm.hip).
constexpr int kCrtConfigs = 3;
// configuration the library picks for an m x n output when none is tuned
int crt_default_config(int64_t m, int64_t n);
// number of moduli for k and s digits, 0 when the product does not fit
int crt_moduli_count(int64_t k, int s);
// One or two levels: N moduli per product, `sets` products (1, or 3 for the
// halves' products hh, ll, ss), the split point (high half's digits) and the
// low half's digit count.  N = 0: not supported.
struct CrtPlan {
    int N, sets, shi, slo;
};
CrtPlan crt_plan(int P, int64_t k, int s);
int crt_products(int P, int64_t k, int s);     // INT8 products of a call, 0 if unsupported
size_t crt_workspace_bytes(int P, int64_t m, int64_t n, int64_t k, int s, int cfg);
int launch_crt(int P, int s, int cfg, const GemmArgs& g, void* ws, hipStream_t st);

// Signatures of the kernel configuration lists a tuning-table entry refers
// to (FNV-1a over each configuration's parameters): plain tiles of precision
// P (also used by the batched form), the split form's tiles, the residue
// form's tiles.
uint32_t fnv1a(uint32_t h, int v);
uint32_t plain_config_signature(int P);
uint32_t split_config_signature();
uint32_t crt_config_signature();

// Residue form over many problems at once (batched plans).  Every problem
// keeps its own workspace region (the single call's layout with 128 x 128
// product tiles); the four stages each run as one launch over all problems,
// a block finding its problem from the per-stage block prefixes b[] (0
// exponents, 1 residues, 2 products, 3 reconstruction).
struct CrtBatchItem {
    GemmArgs g;
    int32_t* E;
    int32_t* F;
    int8_t* RA;
    int8_t* RB;
    uint8_t* Y;
    int64_t Mp, Np, Kp;
    int64_t b[4];
};
// The product stage's blocks on XCD x (block b runs on XCD b % 8) are
// b[2]-indices xcd[x] .. xcd[x + 1] - 1: whole problems, so that the tiles
// sharing a problem's residue panels share that XCD's L2.
struct CrtXcdRanges {
    int64_t xcd[9];
};
struct CrtBatchInfo {
    int N;                 // moduli of every problem (those the largest k needs)
    int sets, shi, slo;    // 1 or 3 products per modulus (two levels: halves of shi, slo digits)
    int mods, groups;      // product stage: planes per workgroup, workgroups per tile
    size_t ws_bytes;       // workspace of all problems
    int64_t blocks[4];     // blocks of each stage (the grid of stages 1, 2, 4)
    CrtXcdRanges ranges;   // product stage
    int64_t grid2;         // its grid: 8 times the most blocks of one XCD
};
// The last item whose first block of stage f is at most bid (the same for
// every lane of the block).
__device__ __forceinline__ int64_t crt_batch_find(const CrtBatchItem* __restrict__ items, int64_t count,
                                                  int64_t bid, int f) {
    int64_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (items[mid].b[f] <= bid) lo = mid; else hi = mid - 1;
    }
    return lo;
}
// Workspace one problem takes in a batch with `planes` residue planes per
// operand (N, or 3N with two levels; a multiple of 256).
size_t crt_batch_item_bytes(int64_t m, int64_t n, int64_t k, int planes);
// Sizes the batch (items == nullptr) or also lays it out in ws and fills
// items (host array of count; problem q goes to XCD q % 8 in the product
// stage, and the items are ordered by XCD, then by q).  pl: the residue
// scheme (crt_plan) of the largest k; problems must be valid with m, n,
// k > 0.  Returns 0, or MPGEMM_ERR_UNSUPPORTED when pl has no moduli or a
// stage's grid would exceed 2^31 - 1 blocks.
int crt_batch_plan(const CrtPlan& pl, int64_t count, const GemmArgs* gs, void* ws, CrtBatchItem* items,
                   CrtBatchInfo* info);
// The four stages on `stream` (d_items: device copy of the items).
int launch_crt_batch(int P, int s, const CrtBatchInfo& info, const CrtBatchItem* d_items, int64_t count,
                     hipStream_t st);
// Stage 1 of a batch: scale exponents of every problem's op(A) rows and
// op(B) columns (split_gemm.hip, beside the single-problem kernels).
int launch_row_exponents_batch(const CrtBatchItem* d_items, int64_t count, int64_t blocks, hipStream_t st);

// The _ex entry points' dispatch for precision P (argument errors numbered as
// for mpgemm_dd_ex, 1..18).
int gemm_ex_entry(int P, char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                  const double* A, int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,
                  const double* beta, double* C, int64_t ldc, int64_t sc, hipStream_t st,
                  const ::mpgemm_opts* opts);
// Its argument checks alone (host only): 0, a negative argument index or
// MPGEMM_ERR_ALIAS.
int gemm_ex_check(int P, char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                  const double* A, int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,
                  const double* beta, double* C, int64_t ldc, int64_t sc, const ::mpgemm_opts* opts);

}  // namespace mpg
