// api.cpp -- the C ABI of libmpgemm (declared in include/mpgemm.h): argument
// validation (host only, before any GPU work), quick returns, form and tile
// dispatch, the batched plan with its captured hipGraph, the autotuner and the
// slice-count rule.
#include "mpgemm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <dlfcn.h>
#include <list>
#include <string>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace mpg {
int launch_axpy(int P, int64_t n, const double* alpha, const double* x, int64_t sx, double* y, int64_t sy,
                hipStream_t st);
size_t dot_workspace_bytes(int P, int64_t n);
int launch_dot(int P, int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* result,
               void* ws, hipStream_t st);
int launch_gemv(int P, int t, int64_t rows, int64_t inner, const double* alpha, const double* A, int64_t lda,
                int64_t sa, const double* x, int64_t sx, const double* beta, double* y, int64_t sy, int az,
                hipStream_t st);
int launch_split_stages(int P, int s, int cfg, int last, const GemmArgs& g, void* ws,
                        hipStream_t st);
int launch_fill(int P, double* X, int64_t plane, int64_t planes_stride, uint64_t seed,
                hipStream_t st);
int launch_absdot(const GemmArgs& g, double* out, hipStream_t st);
int launch_diff_ratio(int P, int64_t m, int64_t n, const double* Cs, const double* Cr, int64_t ld,
                      int64_t ps, const double* absab, double scale, double* out, hipStream_t st);
int launch_probe(int which, double* out, int blocks, int iters, double* ops, hipStream_t st);
int launch_probe_copy(const double* src, double* dst, int64_t n, double* bytes, hipStream_t st);
}  // namespace mpg

using namespace mpg;

namespace {

const int kDefaultSlices[5] = {0, 0, 16, 23, 31};
const int kMaxSlices = 40;
const int kMaxStrassenLevels = 5;

bool valid_trans(char t) {
    return t == 'N' || t == 'n' || t == 'T' || t == 't' || t == 'C' || t == 'c';
}
bool is_trans(char t) { return t != 'N' && t != 'n'; }

bool mp_zero(int P, const double* x) {
    for (int p = 0; p < P; ++p)
        if (x[p] != 0.0) return false;
    return true;
}
bool mp_one(int P, const double* x) {
    if (x[0] != 1.0) return false;
    for (int p = 1; p < P; ++p)
        if (x[p] != 0.0) return false;
    return true;
}

// Byte range [lo, hi) touched by a component-plane matrix.
void extent(const double* X, int P, int64_t rows, int64_t cols, int64_t ld, int64_t ps,
            uintptr_t& lo, uintptr_t& hi) {
    lo = (uintptr_t)X;
    hi = lo + sizeof(double) * (size_t)((P - 1) * ps + (cols - 1) * ld + rows);
}
bool overlaps(uintptr_t a0, uintptr_t a1, uintptr_t b0, uintptr_t b1) { return a0 < b1 && b0 < a1; }

// Validates in signature order; fills g.  Returns 0, a negative argument
// index, or MPGEMM_ERR_ALIAS.
int validate(int P, char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
             const double* A, int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,
             const double* beta, double* C, int64_t ldc, int64_t sc, GemmArgs& g) {
    if (!valid_trans(ta)) return -1;
    if (!valid_trans(tb)) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    if (!alpha) return -6;
    const int64_t nrowa = is_trans(ta) ? k : m, ncola = is_trans(ta) ? m : k;
    const int64_t nrowb = is_trans(tb) ? n : k, ncolb = is_trans(tb) ? k : n;
    const bool reads_ab = m > 0 && n > 0 && k > 0 && !mp_zero(P, alpha);
    if (reads_ab && !A) return -7;
    if (lda < std::max<int64_t>(1, nrowa)) return -8;
    if (sa < lda * ncola) return -9;
    if (reads_ab && !B) return -10;
    if (ldb < std::max<int64_t>(1, nrowb)) return -11;
    if (sb < ldb * ncolb) return -12;
    if (!beta) return -13;
    if (m > 0 && n > 0 && !C) return -14;
    if (ldc < std::max<int64_t>(1, m)) return -15;
    if (sc < ldc * n) return -16;
    if (reads_ab) {
        uintptr_t c0, c1, a0, a1, b0, b1;
        extent(C, P, m, n, ldc, sc, c0, c1);
        extent(A, P, nrowa, ncola, lda, sa, a0, a1);
        extent(B, P, nrowb, ncolb, ldb, sb, b0, b1);
        if (overlaps(c0, c1, a0, a1) || overlaps(c0, c1, b0, b1)) return MPGEMM_ERR_ALIAS;
    }
    g.m = m;
    g.n = n;
    g.k = k;
    g.A = A;
    g.lda = lda;
    g.sa = sa;
    g.B = B;
    g.ldb = ldb;
    g.sb = sb;
    g.C = C;
    g.ldc = ldc;
    g.sc = sc;
    g.ta = is_trans(ta) ? 1 : 0;
    g.tb = is_trans(tb) ? 1 : 0;
    for (int p = 0; p < 4; ++p) {
        g.alpha[p] = p < P ? alpha[p] : 0.0;
        g.beta[p] = p < P ? beta[p] : 0.0;
    }
    return 0;
}

int hip_rc(int e) { return e == 0 ? 0 : MPGEMM_ERR_HIP; }

// ---- tuning table ---------------------------------------------------------

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int>, int> g_tune;
bool g_tune_loaded = false;     // the table file was looked for (first use)

constexpr const char* kTableHeader = "# mpgemm tuning table v2 arch=gfx950";

// The configuration list an entry of form `form` refers to (0 plain, 3
// batched: the plain tiles; 1 split; 5 residue split).
uint32_t config_signature(int P, int form) {
    if (form == MPGEMM_FORM_SPLIT_I8) return split_config_signature();
    if (form == MPGEMM_FORM_SPLIT_CRT) return crt_config_signature();
    return plain_config_signature(P);
}

// Reads a table file into g_tune (lock held).  The first line must be this
// library's header (architecture); an entry is taken only when its
// signature matches the current configuration list of its precision and
// form, so a table written for other kernel configurations is ignored entry
// by entry.  Returns 0, or MPGEMM_ERR_UNSUPPORTED for a file of another
// format or architecture, MPGEMM_ERR_HIP when it cannot be read.
int load_table_locked(const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return MPGEMM_ERR_HIP;
    char line[256];
    int rc = 0;
    if (!std::fgets(line, sizeof line, f) ||
        std::strncmp(line, kTableHeader, std::strlen(kTableHeader)) != 0) {
        rc = MPGEMM_ERR_UNSUPPORTED;
    } else {
        while (std::fgets(line, sizeof line, f)) {
            if (line[0] == '#') continue;
            int P, form, a, b, c, t;
            unsigned sig;
            if (std::sscanf(line, "%d %d %d %d %d %d %x", &P, &form, &a, &b, &c, &t, &sig) != 7) continue;
            if (P < 2 || P > 4 || (form != 0 && form != 1 && form != 3 && form != 5)) continue;
            if (t < 0 || t >= mpgemm_num_configs(P, form) || sig != config_signature(P, form)) continue;
            g_tune[std::make_tuple(P, form, a, b, c)] = t;
        }
    }
    std::fclose(f);
    return rc;
}

// Path of the table shipped beside the shared library.
std::string default_table_path() {
    Dl_info info;
    if (!dladdr((void*)&mpgemm_version, &info) || !info.dli_fname) return std::string();
    std::string so(info.dli_fname);
    const size_t slash = so.rfind('/');
    return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tuned_gfx950.txt";
}

// First use of the table (lock held): load MPGEMM_AUTOTUNE_CACHE, else the
// table beside the library, unless MPGEMM_NO_TUNED_TABLE is set; a missing
// or mismatched file leaves the built-in choices.
void ensure_table_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    if (std::getenv("MPGEMM_NO_TUNED_TABLE")) return;
    const char* env = std::getenv("MPGEMM_AUTOTUNE_CACHE");
    const std::string path = env && *env ? std::string(env) : default_table_path();
    if (!path.empty()) (void)load_table_locked(path.c_str());
}

int ilog2(int64_t x) {
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

int tuned_tile(int P, int form, int64_t m, int64_t n, int64_t k) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_table_locked();
    auto it = g_tune.find(std::make_tuple(P, form, ilog2(m), ilog2(n), ilog2(k)));
    return it == g_tune.end() ? -1 : it->second;
}

int split_default_config(int64_t m, int64_t n) {
    // 64 x 64 tiles, eight diagonals at once, two waves per SIMD: fastest
    // measured at n = 2048 and 4096 (1.6-1.9 POPS); the autotuner may pick
    // another configuration per shape
    (void)m;
    (void)n;
    return 1;
}

int pick_tile(int P, int form, int64_t m, int64_t n, int64_t k, int requested) {
    if (form == MPGEMM_FORM_SPLIT_CRT) {
        if (requested >= 0 && requested < kCrtConfigs) return requested;
        const int t = tuned_tile(P, form, m, n, k);
        if (t >= 0 && t < kCrtConfigs) return t;
        return crt_default_config(m, n);
    }
    const int nconf = form == MPGEMM_FORM_SPLIT_I8 ? kSplitConfigs : kPlainConfigs;
    if (requested >= 0 && requested < nconf) return requested;
    const int t = tuned_tile(P, form, m, n, k);
    if (t >= 0 && t < nconf) return t;
    return form == MPGEMM_FORM_SPLIT_I8 ? split_default_config(m, n)
                                        : plain_default_config(P, m, n, k);
}

bool split_k_ok(int64_t k, int s) { return (int64_t)s * k <= 524287; }

// plain tile for a Strassen bottom block (tuned choice, else the default)
int plain_tile_for(int P, int64_t m, int64_t n, int64_t k) {
    return pick_tile(P, MPGEMM_FORM_PLAIN, m, n, k, -1);
}

bool opts_ok(const mpgemm_opts* opts) {
    if (!opts) return false;
    if (opts->form < 0 || opts->form > 5 || opts->form == 3) return false;
    if (opts->slices < 0 || opts->slices > kMaxSlices) return false;
    if (opts->variant < 0 || opts->variant > 3) return false;
    if (opts->levels < 0 || opts->levels > kMaxStrassenLevels) return false;
    return true;
}

int gemm_common(int P, char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                const double* A, int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,
                const double* beta, double* C, int64_t ldc, int64_t sc, hipStream_t st,
                const mpgemm_opts* opts, bool has_opts, int last_stage) {
    GemmArgs g;
    int rc = validate(P, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, g);
    if (rc) return rc;
    if (has_opts && !opts_ok(opts)) return -18;
    const int variant = has_opts ? opts->variant : 0;
    // the TD variants exist for the plain form only
    if (variant != 0 && (P != 3 || opts->form == MPGEMM_FORM_SPLIT_I8 ||
                         opts->form == MPGEMM_FORM_STRASSEN || opts->form == MPGEMM_FORM_SPLIT_CRT ||
                         last_stage > 0))
        return MPGEMM_ERR_UNSUPPORTED;
    const bool strassen = has_opts && opts->form == MPGEMM_FORM_STRASSEN && last_stage <= 0;
    const int levels = strassen ? (opts->levels > 0 ? opts->levels : 1) : 0;
    if (strassen) {
        const int64_t unit = (int64_t)1 << levels;
        if (m % unit || n % unit || k % unit) return MPGEMM_ERR_UNSUPPORTED;
    }
    const bool crt = has_opts && opts->form == MPGEMM_FORM_SPLIT_CRT && last_stage <= 0;
    const int crt_s = crt ? (opts->slices > 0 ? opts->slices : kDefaultSlices[P]) : 0;
    // the residue form needs enough moduli for the exact product (checked
    // for every shape, also those that return early)
    if (crt && k > 0 && crt_products(P, k, crt_s) == 0) return MPGEMM_ERR_UNSUPPORTED;
    if (m == 0 || n == 0) return 0;
    const bool az = (k == 0) || mp_zero(P, alpha);
    if (az && mp_one(P, beta)) return 0;
    if (az) return hip_rc(variant ? launch_scale_td_variant(variant, g, st) : launch_scale(P, g, st));
    if (variant) return hip_rc(launch_plain_td_variant(variant, g, st));
    if (strassen) {
        const size_t need = strassen_workspace_bytes(P, levels, m, n, k);
        if (!opts->workspace || opts->workspace_bytes < need) return MPGEMM_ERR_WORKSPACE;
        if ((uintptr_t)opts->workspace % 256 != 0) return MPGEMM_ERR_WORKSPACE;
        return hip_rc(launch_strassen(P, levels, g, opts->workspace, st, &plain_tile_for));
    }
    if (crt) {
        const int cfg = pick_tile(P, MPGEMM_FORM_SPLIT_CRT, m, n, k, opts->tile);
        const size_t need = crt_workspace_bytes(P, m, n, k, crt_s, cfg);
        if (!opts->workspace || opts->workspace_bytes < need) return MPGEMM_ERR_WORKSPACE;
        if ((uintptr_t)opts->workspace % 256 != 0) return MPGEMM_ERR_WORKSPACE;
        return hip_rc(launch_crt(P, crt_s, cfg, g, opts->workspace, st));
    }

    int form = has_opts ? opts->form : MPGEMM_FORM_PLAIN;
    const int s = (has_opts && opts->slices > 0) ? opts->slices : kDefaultSlices[P];
    const int req_tile = has_opts ? opts->tile : -1;
    if (last_stage > 0) form = MPGEMM_FORM_SPLIT_I8;
    // the split forms' error grows with the spread of magnitudes within a
    // row of op(A) or a column of op(B), which the call cannot see without
    // reading the operands; the library takes them only when the caller has
    // chosen the digit count (for example with mpgemm_tune_slices)
    if (form == MPGEMM_FORM_AUTO && opts->slices == 0) form = MPGEMM_FORM_PLAIN;
    // the residue form's smallest sizes, measured: from 128 (DD), 96 (TD) and
    // 64 (QD) in every dimension it beats the plain and the triangular forms
    const int64_t crt_min = P == 2 ? 128 : (P == 3 ? 96 : 64);
    if (form == MPGEMM_FORM_AUTO && m >= crt_min && n >= crt_min && k >= crt_min && opts->workspace &&
        (uintptr_t)opts->workspace % 256 == 0 && crt_products(P, k, s) > 0) {
        // the residue form first: the fastest split variant wherever it applies
        const int cfg = pick_tile(P, MPGEMM_FORM_SPLIT_CRT, m, n, k, req_tile);
        if (opts->workspace_bytes >= crt_workspace_bytes(P, m, n, k, s, cfg))
            return hip_rc(launch_crt(P, s, cfg, g, opts->workspace, st));
    }
    if (form == MPGEMM_FORM_AUTO) {
        // a workspace that cannot hold the split form (too small or not
        // 256-byte aligned) means plain, not an error
        const bool fits = opts->workspace && (uintptr_t)opts->workspace % 256 == 0 &&
                          opts->workspace_bytes >= split_workspace_bytes(
                              P, m, n, k, s, pick_tile(P, MPGEMM_FORM_SPLIT_I8, m, n, k, req_tile));
        form = (fits && split_k_ok(k, s) && m >= 256 && n >= 256 && k >= 256)
                   ? MPGEMM_FORM_SPLIT_I8 : MPGEMM_FORM_PLAIN;
    }
    if (form == MPGEMM_FORM_PLAIN) {
        const int cfg = pick_tile(P, form, m, n, k, req_tile);
        return hip_rc(launch_plain(P, cfg, g, st));
    }
    if (!split_k_ok(k, s)) return MPGEMM_ERR_UNSUPPORTED;
    const int cfg = pick_tile(P, MPGEMM_FORM_SPLIT_I8, m, n, k, req_tile);
    const size_t need = split_workspace_bytes(P, m, n, k, s, cfg);
    if (!opts->workspace || opts->workspace_bytes < need) return MPGEMM_ERR_WORKSPACE;
    if ((uintptr_t)opts->workspace % 256 != 0) return MPGEMM_ERR_WORKSPACE;
    return hip_rc(launch_split_stages(P, s, cfg, last_stage > 0 ? last_stage : 4, g, opts->workspace, st));
}

}  // namespace

// ===========================================================================
extern "C" {

#define MPG_GEMM(NAME, P)                                                                          \
    int NAME(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,              \
             const double* A, int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,  \
             const double* beta, double* C, int64_t ldc, int64_t sc, hipStream_t st) {            \
        return gemm_common(P, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, st, \
                           nullptr, false, 0);                                                    \
    }                                                                                              \
    int NAME##_ex(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,         \
                  const double* A, int64_t lda, int64_t sa, const double* B, int64_t ldb,          \
                  int64_t sb, const double* beta, double* C, int64_t ldc, int64_t sc,             \
                  hipStream_t st, const mpgemm_opts* opts) {                                       \
        return gemm_common(P, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, st, \
                           opts, true, 0);                                                        \
    }

MPG_GEMM(mpgemm_dd, 2)
MPG_GEMM(mpgemm_td, 3)
MPG_GEMM(mpgemm_qd, 4)
#undef MPG_GEMM
}  // extern "C"

namespace mpg {
int gemm_ex_entry(int P, char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                  const double* A, int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,
                  const double* beta, double* C, int64_t ldc, int64_t sc, hipStream_t st,
                  const mpgemm_opts* opts) {
    return gemm_common(P, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, st, opts,
                       true, 0);
}

int gemm_ex_check(int P, char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                  const double* A, int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,
                  const double* beta, double* C, int64_t ldc, int64_t sc, const mpgemm_opts* opts) {
    GemmArgs g;
    const int rc = validate(P, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, g);
    if (rc) return rc;
    return opts_ok(opts) ? 0 : -18;
}
}  // namespace mpg

extern "C" {

size_t mpgemm_workspace_bytes(int prec, int form, int64_t m, int64_t n, int64_t k, int slices,
                              int tile) {
    if (prec < 2 || prec > 4 || m < 0 || n < 0 || k < 0 || slices < 0 || slices > kMaxSlices)
        return 0;
    if (form == MPGEMM_FORM_PLAIN) return 0;
    if (form == MPGEMM_FORM_STRASSEN) {
        const int levels = slices > 0 ? slices : 1;
        if (levels > kMaxStrassenLevels) return 0;
        return strassen_workspace_bytes(prec, levels, m, n, k);
    }
    if (form == MPGEMM_FORM_SPLIT_CRT) {
        const int s = slices > 0 ? slices : kDefaultSlices[prec];
        return crt_workspace_bytes(prec, m, n, k, s, pick_tile(prec, form, m, n, k, tile));
    }
    if (form != MPGEMM_FORM_SPLIT_I8 && form != MPGEMM_FORM_AUTO) return 0;
    const int s = slices > 0 ? slices : kDefaultSlices[prec];
    const int cfg = pick_tile(prec, MPGEMM_FORM_SPLIT_I8, m, n, k, tile);
    const size_t split = split_workspace_bytes(prec, m, n, k, s, cfg);
    if (form == MPGEMM_FORM_AUTO && crt_products(prec, k, s) > 0) {
        // room for either split variant
        const size_t crt = crt_workspace_bytes(prec, m, n, k, s, pick_tile(prec, MPGEMM_FORM_SPLIT_CRT, m, n, k, tile));
        return crt > split ? crt : split;
    }
    return split;
}

int mpgemm_crt_moduli(int prec, int64_t k, int slices) {
    if (prec < 2 || prec > 4) return -1;
    if (slices < 0 || slices > kMaxSlices) return 0;
    return crt_products(prec, k, slices > 0 ? slices : kDefaultSlices[prec]);
}

int mpgemm_split_layout(int prec, int64_t m, int64_t n, int64_t k, int slices, int tile,
                        size_t* off_E, size_t* off_F, size_t* off_DA, size_t* off_DB,
                        size_t* off_S, int64_t* Mp, int64_t* Np, int64_t* Kp) {
    if (prec < 2 || prec > 4) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (k < 0) return -4;
    if (slices < 0 || slices > kMaxSlices) return -5;
    const int s = slices > 0 ? slices : kDefaultSlices[prec];
    const int cfg = pick_tile(prec, MPGEMM_FORM_SPLIT_I8, m, n, k, tile);
    if (!off_E || !off_F || !off_DA || !off_DB || !off_S || !Mp || !Np || !Kp) return -7;
    return split_layout(prec, m, n, k, s, cfg, off_E, off_F, off_DA, off_DB, off_S, Mp, Np, Kp);
}

int mpgemm_split_stages(int prec, int last, char ta, char tb, int64_t m, int64_t n, int64_t k,
                        const double* alpha, const double* A, int64_t lda, int64_t sa,
                        const double* B, int64_t ldb, int64_t sb, const double* beta, double* C,
                        int64_t ldc, int64_t sc, hipStream_t st, const mpgemm_opts* opts) {
    if (prec < 2 || prec > 4) return -1;
    if (last < 1 || last > 4) return -2;
    int rc = gemm_common(prec, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, st,
                         opts, true, last);
    // re-number argument errors of the shared part (shifted by the two leading args)
    return rc < 0 ? rc - 2 : rc;
}

#define MPG_VEC(NAME, P, OP)                                                                     \
    int NAME(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* r,     \
             int64_t sr, hipStream_t st) {                                                       \
        if (n < 0) return -1;                                                                    \
        if (n > 0 && !x) return -2;                                                              \
        if (sx < n) return -3;                                                                   \
        if (n > 0 && !y) return -4;                                                              \
        if (sy < n) return -5;                                                                   \
        if (n > 0 && !r) return -6;                                                              \
        if (sr < n) return -7;                                                                   \
        if (n == 0) return 0;                                                                    \
        return hip_rc(launch_vec(P, OP, n, x, sx, y, sy, r, sr, st));                            \
    }
MPG_VEC(mp_vec_dd_add, 2, 0)
MPG_VEC(mp_vec_dd_mul, 2, 1)
MPG_VEC(mp_vec_td_add, 3, 0)
MPG_VEC(mp_vec_td_mul, 3, 1)
MPG_VEC(mp_vec_qd_add, 4, 0)
MPG_VEC(mp_vec_qd_mul, 4, 1)
MPG_VEC(mp_vec_td_add_acc, 3, 2)
MPG_VEC(mp_vec_td_mulq, 3, 3)
#undef MPG_VEC

// ---- BLAS-1/2 ----------------------------------------------------------------

#define MPG_AXPY(NAME, P)                                                                          \
    int NAME(int64_t n, const double* alpha, const double* x, int64_t sx, double* y, int64_t sy,  \
             hipStream_t st) {                                                                    \
        if (n < 0) return -1;                                                                      \
        if (!alpha) return -2;                                                                     \
        if (n > 0 && !x) return -3;                                                                \
        if (sx < n) return -4;                                                                     \
        if (n > 0 && !y) return -5;                                                                \
        if (sy < n) return -6;                                                                     \
        return hip_rc(launch_axpy(P, n, alpha, x, sx, y, sy, st));                                 \
    }
MPG_AXPY(mp_axpy_dd, 2)
MPG_AXPY(mp_axpy_td, 3)
MPG_AXPY(mp_axpy_qd, 4)
#undef MPG_AXPY

size_t mp_dot_workspace_bytes(int prec, int64_t n) {
    if (prec < 2 || prec > 4 || n < 0) return 0;
    return dot_workspace_bytes(prec, n);
}

#define MPG_DOT(NAME, P)                                                                           \
    int NAME(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* result,  \
             void* ws, size_t ws_bytes, hipStream_t st) {                                          \
        if (n < 0) return -1;                                                                      \
        if (n > 0 && !x) return -2;                                                                \
        if (sx < n) return -3;                                                                     \
        if (n > 0 && !y) return -4;                                                                \
        if (sy < n) return -5;                                                                     \
        if (!result) return -6;                                                                    \
        const size_t need = dot_workspace_bytes(P, n);                                             \
        if (need > 0 && !ws) return -7;                                                            \
        if (ws_bytes < need) return MPGEMM_ERR_WORKSPACE;                                          \
        return hip_rc(launch_dot(P, n, x, sx, y, sy, result, ws, st));                             \
    }
MPG_DOT(mp_dot_dd, 2)
MPG_DOT(mp_dot_td, 3)
MPG_DOT(mp_dot_qd, 4)
#undef MPG_DOT

static int gemv_common(int P, char trans, int64_t m, int64_t n, const double* alpha, const double* A,
                       int64_t lda, int64_t sa, const double* x, int64_t sx, const double* beta, double* y,
                       int64_t sy, hipStream_t st) {
    if (!valid_trans(trans)) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (!alpha) return -4;
    const int t = is_trans(trans) ? 1 : 0;
    const int64_t rows = t ? n : m, inner = t ? m : n;
    const bool az = mp_zero(P, alpha) || inner == 0;
    const bool reads_a = rows > 0 && !az;
    if (reads_a && !A) return -5;
    if (lda < std::max<int64_t>(1, m)) return -6;
    if (sa < lda * n) return -7;
    if (reads_a && !x) return -8;
    if (sx < inner) return -9;
    if (!beta) return -10;
    if (rows > 0 && !y) return -11;
    if (sy < rows) return -12;
    if (rows == 0 || (az && mp_one(P, beta))) return 0;
    if (reads_a) {
        uintptr_t y0, y1, a0, a1, x0, x1;
        extent(y, P, rows, 1, rows, sy, y0, y1);
        extent(A, P, m, n, lda, sa, a0, a1);
        extent(x, P, inner, 1, inner, sx, x0, x1);
        if (overlaps(y0, y1, a0, a1) || overlaps(y0, y1, x0, x1)) return MPGEMM_ERR_ALIAS;
    }
    return hip_rc(launch_gemv(P, t, rows, inner, alpha, A, lda, sa, x, sx, beta, y, sy, az ? 1 : 0, st));
}

#define MPG_GEMV(NAME, P)                                                                           \
    int NAME(char trans, int64_t m, int64_t n, const double* alpha, const double* A, int64_t lda,     \
             int64_t sa, const double* x, int64_t sx, const double* beta, double* y, int64_t sy,      \
             hipStream_t st) {                                                                       \
        return gemv_common(P, trans, m, n, alpha, A, lda, sa, x, sx, beta, y, sy, st);               \
    }
MPG_GEMV(mp_gemv_dd, 2)
MPG_GEMV(mp_gemv_td, 3)
MPG_GEMV(mp_gemv_qd, 4)
#undef MPG_GEMV

// ---- batched plan -----------------------------------------------------------

// Residue problems of a plan run in chunks whose workspace stays within a
// bound (opts->workspace_bytes, else this default; a problem larger than it
// forms a chunk of its own); the chunks run one after another on the plan's
// stream and share one workspace.
constexpr size_t kBatchChunkBytes = (size_t)8 << 30;

struct CrtChunk {
    int64_t first, count;     // items first .. first + count - 1
    CrtBatchInfo info;
};

struct mpgemm_batch_plan {
    int P;
    int cfg;
    int64_t count;            // problems of the plain part
    int64_t tiles;
    int grid;
    void* d_desc;
    unsigned* d_counter;
    int crt_s;                // residue part: digits, problems, chunks
    int64_t crt_count;
    std::vector<CrtChunk> chunks;
    CrtBatchItem* d_items;
    void* d_ws;
    size_t ws_bytes;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

int plan_launch_all(const mpgemm_batch_plan* plan, hipStream_t st) {
    if (plan->tiles > 0) {
        const int rc = launch_batch(plan->P, plan->cfg, plan->count, plan->tiles, plan->d_desc, plan->d_counter,
                                    plan->grid, st);
        if (rc) return rc;
    }
    for (const CrtChunk& c : plan->chunks) {
        const int rc = launch_crt_batch(plan->P, plan->crt_s, c.info, plan->d_items + c.first, c.count, st);
        if (rc) return rc;
    }
    return 0;
}

bool plan_empty(const mpgemm_batch_plan* plan) { return plan->tiles == 0 && plan->chunks.empty(); }

// The residue part: chunks laid out over one workspace, items copied to the
// device (synchronously on st).  gs: the residue problems, largest first.
int plan_residue_part(mpgemm_batch_plan* plan, const CrtPlan& pl, int s, size_t bound,
                      const std::vector<GemmArgs>& gs, hipStream_t st) {
    const int64_t cnt = (int64_t)gs.size();
    plan->crt_s = s;
    plan->crt_count = cnt;
    // chunks: consecutive problems while their workspace fits the bound
    std::vector<std::pair<int64_t, int64_t>> ranges;
    size_t ws = 0, cur = 0;
    int64_t first = 0;
    for (int64_t q = 0; q < cnt; ++q) {
        const size_t b = crt_batch_item_bytes(gs[(size_t)q].m, gs[(size_t)q].n, gs[(size_t)q].k, pl.N * pl.sets);
        if (q > first && cur + b > bound) {
            ranges.emplace_back(first, q - first);
            first = q;
            cur = 0;
        }
        cur += b;
        ws = std::max(ws, cur);
    }
    if (cnt > 0) ranges.emplace_back(first, cnt - first);
    if (hipMalloc(&plan->d_ws, std::max<size_t>(ws, 256)) != hipSuccess) return MPGEMM_ERR_NOMEM;
    plan->ws_bytes = ws;
    const size_t ibytes = sizeof(CrtBatchItem) * (size_t)std::max<int64_t>(cnt, 1);
    if (hipMalloc((void**)&plan->d_items, ibytes) != hipSuccess) return MPGEMM_ERR_NOMEM;
    std::vector<CrtBatchItem> items((size_t)std::max<int64_t>(cnt, 1));
    for (const auto& r : ranges) {
        CrtChunk c{r.first, r.second, {}};
        const int rc = crt_batch_plan(pl, c.count, gs.data() + c.first, plan->d_ws, items.data() + c.first, &c.info);
        if (rc) return rc;
        plan->chunks.push_back(c);
    }
    if (hipMemcpyAsync(plan->d_items, items.data(), ibytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MPGEMM_ERR_HIP;
    return 0;
}

}  // namespace

int mpgemm_batch_plan_create(int prec, int64_t count, const mpgemm_problem* probs,
                             const mpgemm_opts* opts, hipStream_t st, mpgemm_batch_plan** out) {
    if (prec < 2 || prec > 4) return -1;
    if (count < 0) return -2;
    if (count > 0 && !probs) return -3;
    if (!out) return -6;
    *out = nullptr;
    if (opts && !opts_ok(opts)) return -4;
    const int P = prec;
    std::vector<GemmArgs> gs((size_t)count);
    for (int64_t q = 0; q < count; ++q) {
        const mpgemm_problem& pr = probs[q];
        int rc = validate(P, pr.transa, pr.transb, pr.m, pr.n, pr.k, pr.alpha, pr.A, pr.lda,
                          pr.a_plane_stride, pr.B, pr.ldb, pr.b_plane_stride, pr.beta, pr.C,
                          pr.ldc, pr.c_plane_stride, gs[(size_t)q]);
        if (rc) return rc == MPGEMM_ERR_ALIAS ? rc : (int)(-(1000 + q));
    }
    if (opts && opts->variant != 0) return MPGEMM_ERR_UNSUPPORTED;   // TD variants: plain calls only
    const int form = opts ? opts->form : MPGEMM_FORM_PLAIN;
    if (form != MPGEMM_FORM_PLAIN && form != MPGEMM_FORM_AUTO && form != MPGEMM_FORM_SPLIT_CRT)
        return MPGEMM_ERR_UNSUPPORTED;
    // which problems take the residue form: all that multiply (SPLIT_CRT), or
    // with s given those of at least the single call's residue sizes (AUTO)
    const int s = (opts && opts->slices > 0) ? opts->slices : kDefaultSlices[P];
    const int64_t crt_min = P == 2 ? 128 : (P == 3 ? 96 : 64);
    std::vector<char> res((size_t)count, 0);
    int64_t kmax = 0;
    for (int64_t q = 0; q < count; ++q) {
        const GemmArgs& g = gs[(size_t)q];
        const bool mult = g.m > 0 && g.n > 0 && g.k > 0 && !mp_zero(P, g.alpha);
        bool r = false;
        if (form == MPGEMM_FORM_SPLIT_CRT && mult) {
            if (crt_plan(P, g.k, s).N == 0) return MPGEMM_ERR_UNSUPPORTED;
            r = true;
        } else if (form == MPGEMM_FORM_AUTO && mult && opts->slices > 0) {
            r = g.m >= crt_min && g.n >= crt_min && g.k >= crt_min && crt_plan(P, g.k, s).N > 0;
        }
        res[(size_t)q] = r;
        if (r) kmax = std::max(kmax, g.k);
    }
    std::vector<GemmArgs> gp, gr;
    for (int64_t q = 0; q < count; ++q) (res[(size_t)q] ? gr : gp).push_back(gs[(size_t)q]);
    const int64_t np = (int64_t)gp.size();

    int cfg = (opts && opts->tile >= 0 && opts->tile < kPlainConfigs) ? opts->tile : -1;
    if (cfg < 0) {
        // tile shape for the typical problem of the plain part
        int64_t mm = 0, nn = 0, kk = 0;
        for (const auto& g : gp) { mm += g.m; nn += g.n; kk += g.k; }
        if (np > 0) { mm /= np; nn /= np; kk /= np; }
        cfg = tuned_tile(P, 3, mm, nn, kk);      // form id 3: batched
        // untuned: the tiles measured fastest on 512 problems with m, n, k
        // uniform in [16, 512] (DD 64 x 32, TD and QD 16 x 16)
        if (cfg < 0) cfg = P == 2 ? 2 : 3;
    }
    // largest k first so the queue ends with the cheapest tiles
    std::vector<int64_t> order((size_t)np);
    for (int64_t q = 0; q < np; ++q) order[(size_t)q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return gp[(size_t)a].k > gp[(size_t)b].k;
    });
    // residue problems: the largest first, so that the last blocks of each
    // stage are the small ones
    std::stable_sort(gr.begin(), gr.end(), [](const GemmArgs& a, const GemmArgs& b) {
        return (double)a.m * a.n * a.k > (double)b.m * b.n * b.k;
    });
    auto* plan = new (std::nothrow) mpgemm_batch_plan();
    if (!plan) return MPGEMM_ERR_NOMEM;
    plan->P = P;
    plan->cfg = cfg;
    plan->count = np;
    const size_t bytes = std::max<size_t>(batch_desc_bytes(np), 256);
    std::vector<char> host(bytes);
    plan->tiles = batch_build_desc(P, cfg, np, gp.data(), order.data(), host.data());
    plan->grid = (int)std::max<int64_t>(1, std::min<int64_t>(batch_max_grid(P, cfg), plan->tiles));
    int err = 0;
    if (hipMalloc(&plan->d_desc, bytes) != hipSuccess || hipMalloc((void**)&plan->d_counter, 256) != hipSuccess)
        err = MPGEMM_ERR_NOMEM;
    if (!err && (hipMemcpyAsync(plan->d_desc, host.data(), bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
                 hipStreamSynchronize(st) != hipSuccess))
        err = MPGEMM_ERR_HIP;
    const size_t bound = (opts && opts->workspace_bytes > 0) ? opts->workspace_bytes : kBatchChunkBytes;
    if (!err && !gr.empty()) err = plan_residue_part(plan, crt_plan(P, kmax, s), s, bound, gr, st);
    // capture every launch of a run on a private stream
    hipStream_t cs = nullptr;
    if (!err && !plan_empty(plan)) {
        if (hipStreamCreate(&cs) != hipSuccess) err = MPGEMM_ERR_GRAPH;
        else {
            if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) err = MPGEMM_ERR_GRAPH;
            else {
                const int lrc = plan_launch_all(plan, cs);
                hipGraph_t graph = nullptr;
                if (hipStreamEndCapture(cs, &graph) != hipSuccess || lrc) err = MPGEMM_ERR_GRAPH;
                plan->graph = graph;
                if (!err && hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0) != hipSuccess)
                    err = MPGEMM_ERR_GRAPH;
            }
            (void)hipStreamDestroy(cs);
        }
    }
    if (err) {
        mpgemm_batch_plan_destroy(plan);
        return err;
    }
    *out = plan;
    return 0;
}

int mpgemm_batch_plan_run(mpgemm_batch_plan* plan, hipStream_t st) {
    if (!plan) return -1;
    if (plan_empty(plan)) return 0;
    return hipGraphLaunch(plan->exec, st) == hipSuccess ? 0 : MPGEMM_ERR_HIP;
}

int mpgemm_batch_plan_launch(mpgemm_batch_plan* plan, hipStream_t st) {
    if (!plan) return -1;
    return hip_rc(plan_launch_all(plan, st));
}

int mpgemm_batch_plan_info(const mpgemm_batch_plan* plan, int64_t* tiles, int* grid, int* tile_cfg) {
    if (!plan) return -1;
    if (tiles) *tiles = plan->tiles;
    if (grid) *grid = plan->grid;
    if (tile_cfg) *tile_cfg = plan->cfg;
    return 0;
}

int mpgemm_batch_plan_residue_info(const mpgemm_batch_plan* plan, int64_t* problems, int* moduli, int* chunks,
                                   size_t* workspace_bytes) {
    if (!plan) return -1;
    if (problems) *problems = plan->crt_count;
    if (moduli) *moduli = plan->chunks.empty() ? 0 : plan->chunks[0].info.N * plan->chunks[0].info.sets;
    if (chunks) *chunks = (int)plan->chunks.size();
    if (workspace_bytes) *workspace_bytes = plan->ws_bytes;
    return 0;
}

int mpgemm_batch_plan_destroy(mpgemm_batch_plan* plan) {
    if (!plan) return -1;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->d_desc) (void)hipFree(plan->d_desc);
    if (plan->d_counter) (void)hipFree(plan->d_counter);
    if (plan->d_items) (void)hipFree(plan->d_items);
    if (plan->d_ws) (void)hipFree(plan->d_ws);
    delete plan;
    return 0;
}

// ---- grouped calls: plans cached by problem array ----------------------------

}  // extern "C"

namespace {

struct GroupedPlan {
    int P, tile, form, slices;
    std::vector<mpgemm_problem> probs;
    mpgemm_batch_plan* plan;
};
std::mutex g_group_mu;
std::list<GroupedPlan> g_groups;          // most recently used first
constexpr size_t kMaxGroupedPlans = 8;

bool same_double(double a, double b) { return std::memcmp(&a, &b, sizeof a) == 0; }

// Field by field (the struct's padding bytes are not compared).
bool same_problem(int P, const mpgemm_problem& a, const mpgemm_problem& b) {
    if (a.transa != b.transa || a.transb != b.transb || a.m != b.m || a.n != b.n || a.k != b.k) return false;
    for (int p = 0; p < P; ++p)
        if (!same_double(a.alpha[p], b.alpha[p]) || !same_double(a.beta[p], b.beta[p])) return false;
    return a.A == b.A && a.lda == b.lda && a.a_plane_stride == b.a_plane_stride && a.B == b.B &&
           a.ldb == b.ldb && a.b_plane_stride == b.b_plane_stride && a.C == b.C && a.ldc == b.ldc &&
           a.c_plane_stride == b.c_plane_stride;
}

int grouped_common(int P, int64_t count, const mpgemm_problem* probs, const mpgemm_opts* opts,
                    hipStream_t st) {
    if (count < 0) return -1;
    if (count > 0 && !probs) return -2;
    if (opts && (!opts_ok(opts) ||
                 (opts->form != MPGEMM_FORM_PLAIN && opts->form != MPGEMM_FORM_AUTO &&
                  opts->form != MPGEMM_FORM_SPLIT_CRT) ||
                 opts->variant != 0))
        return -3;
    if (count == 0) return 0;
    const int tile = (opts && opts->tile >= 0 && opts->tile < kPlainConfigs) ? opts->tile : -1;
    const int form = opts ? opts->form : MPGEMM_FORM_PLAIN, slices = opts ? opts->slices : 0;
    std::lock_guard<std::mutex> lk(g_group_mu);
    for (auto it = g_groups.begin(); it != g_groups.end(); ++it) {
        if (it->P != P || it->tile != tile || it->form != form || it->slices != slices ||
            (int64_t)it->probs.size() != count)
            continue;
        bool same = true;
        for (int64_t q = 0; q < count && same; ++q) same = same_problem(P, it->probs[(size_t)q], probs[q]);
        if (!same) continue;
        g_groups.splice(g_groups.begin(), g_groups, it);
        return mpgemm_batch_plan_run(g_groups.front().plan, st);
    }
    mpgemm_opts o{};
    o.tile = tile;
    o.form = form;
    o.slices = slices;
    mpgemm_batch_plan* plan = nullptr;
    const int rc = mpgemm_batch_plan_create(P, count, probs, &o, st, &plan);
    if (rc) return rc;
    if (g_groups.size() >= kMaxGroupedPlans) {
        // the least recently used plan may still run on some stream
        if (hipDeviceSynchronize() != hipSuccess) {
            (void)mpgemm_batch_plan_destroy(plan);
            return MPGEMM_ERR_HIP;
        }
        (void)mpgemm_batch_plan_destroy(g_groups.back().plan);
        g_groups.pop_back();
    }
    g_groups.push_front(GroupedPlan{P, tile, form, slices, std::vector<mpgemm_problem>(probs, probs + count), plan});
    return mpgemm_batch_plan_run(plan, st);
}

void release_grouped_plans() {
    std::lock_guard<std::mutex> lk(g_group_mu);
    if (!g_groups.empty()) (void)hipDeviceSynchronize();
    for (auto& g : g_groups) (void)mpgemm_batch_plan_destroy(g.plan);
    g_groups.clear();
}

}  // namespace

extern "C" {

int mpgemm_dd_grouped(int64_t count, const mpgemm_problem* problems, const mpgemm_opts* opts,
                      hipStream_t stream) {
    return grouped_common(2, count, problems, opts, stream);
}
int mpgemm_td_grouped(int64_t count, const mpgemm_problem* problems, const mpgemm_opts* opts,
                      hipStream_t stream) {
    return grouped_common(3, count, problems, opts, stream);
}
int mpgemm_qd_grouped(int64_t count, const mpgemm_problem* problems, const mpgemm_opts* opts,
                      hipStream_t stream) {
    return grouped_common(4, count, problems, opts, stream);
}

// ---- autotuner --------------------------------------------------------------

int mpgemm_num_configs(int prec, int form) {
    if (prec < 2 || prec > 4) return 0;
    if (form == MPGEMM_FORM_PLAIN || form == 3) return kPlainConfigs;
    if (form == MPGEMM_FORM_SPLIT_I8) return kSplitConfigs;
    if (form == MPGEMM_FORM_SPLIT_CRT) return kCrtConfigs;
    return 0;
}

static int time_config(int P, int form, int cfg, const GemmArgs& g, int s, void* ws, size_t wsb,
                       hipStream_t st, float* ms_out) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MPGEMM_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return MPGEMM_ERR_HIP; }
    auto run = [&]() {
        return form == MPGEMM_FORM_PLAIN     ? launch_plain(P, cfg, g, st)
               : form == MPGEMM_FORM_SPLIT_CRT ? launch_crt(P, s, cfg, g, ws, st)
                                               : launch_split(P, s, cfg, g, ws, wsb, st);
    };
    int rc = run();  // warm-up
    float best = 1e30f;
    for (int rep = 0; rep < 3 && !rc; ++rep) {
        (void)hipEventRecord(e0, st);
        rc = run();
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) rc = MPGEMM_ERR_HIP;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = best;
    return rc ? MPGEMM_ERR_HIP : 0;
}

int mpgemm_autotune(int prec, int form, int64_t m, int64_t n, int64_t k, int slices,
                    hipStream_t st, int* best) {
    if (prec < 2 || prec > 4) return -1;
    if (form != MPGEMM_FORM_PLAIN && form != MPGEMM_FORM_SPLIT_I8 && form != MPGEMM_FORM_SPLIT_CRT)
        return -2;
    if (m <= 0) return -3;
    if (n <= 0) return -4;
    if (k <= 0) return -5;
    if (slices < 0 || slices > kMaxSlices) return -6;
    const int P = prec;
    const int s = slices > 0 ? slices : kDefaultSlices[P];
    if (form == MPGEMM_FORM_SPLIT_I8 && !split_k_ok(k, s)) return MPGEMM_ERR_UNSUPPORTED;
    if (form == MPGEMM_FORM_SPLIT_CRT && crt_products(P, k, s) == 0) return MPGEMM_ERR_UNSUPPORTED;
    double *A = nullptr, *B = nullptr, *C = nullptr;
    void* ws = nullptr;
    size_t wsb = 0;
    const size_t na = (size_t)P * m * k, nb = (size_t)P * k * n, nc = (size_t)P * m * n;
    int rc = 0;
    if (hipMalloc((void**)&A, na * 8) != hipSuccess || hipMalloc((void**)&B, nb * 8) != hipSuccess ||
        hipMalloc((void**)&C, nc * 8) != hipSuccess)
        rc = MPGEMM_ERR_NOMEM;
    if (!rc && form == MPGEMM_FORM_SPLIT_I8) {
        for (int c = 0; c < kSplitConfigs; ++c) wsb = std::max(wsb, split_workspace_bytes(P, m, n, k, s, c));
        if (hipMalloc(&ws, wsb) != hipSuccess) rc = MPGEMM_ERR_NOMEM;
    }
    if (!rc && form == MPGEMM_FORM_SPLIT_CRT) {
        for (int c = 0; c < kCrtConfigs; ++c) wsb = std::max(wsb, crt_workspace_bytes(P, m, n, k, s, c));
        if (hipMalloc(&ws, wsb) != hipSuccess) rc = MPGEMM_ERR_NOMEM;
    }
    if (!rc) rc = launch_fill(P, A, m * k, m * k, 11, st) ? MPGEMM_ERR_HIP : 0;
    if (!rc) rc = launch_fill(P, B, k * n, k * n, 12, st) ? MPGEMM_ERR_HIP : 0;
    int chosen = -1;
    if (!rc) {
        GemmArgs g{};
        g.m = m; g.n = n; g.k = k;
        g.A = A; g.lda = m; g.sa = m * k;
        g.B = B; g.ldb = k; g.sb = k * n;
        g.C = C; g.ldc = m; g.sc = m * n;
        g.alpha[0] = 1.0;
        float best_ms = 1e30f;
        const int nconf = mpgemm_num_configs(P, form);
        for (int c = 0; c < nconf && !rc; ++c) {
            float ms = 0.f;
            rc = time_config(P, form, c, g, s, ws, wsb, st, &ms);
            if (!rc && ms < best_ms) { best_ms = ms; chosen = c; }
        }
    }
    if (A) (void)hipFree(A);
    if (B) (void)hipFree(B);
    if (C) (void)hipFree(C);
    if (ws) (void)hipFree(ws);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        ensure_table_locked();
        g_tune[std::make_tuple(P, form, ilog2(m), ilog2(n), ilog2(k))] = chosen;
    }
    if (best) *best = chosen;
    return 0;
}

int mpgemm_autotune_set(int prec, int form, int64_t m, int64_t n, int64_t k, int tile) {
    if (prec < 2 || prec > 4) return -1;
    if (form != MPGEMM_FORM_PLAIN && form != MPGEMM_FORM_SPLIT_I8 && form != MPGEMM_FORM_SPLIT_CRT &&
        form != 3)
        return -2;
    if (m <= 0) return -3;
    if (n <= 0) return -4;
    if (k <= 0) return -5;
    if (tile < 0 || tile >= mpgemm_num_configs(prec, form)) return -6;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_table_locked();
    g_tune[std::make_tuple(prec, form, ilog2(m), ilog2(n), ilog2(k))] = tile;
    return 0;
}

int mpgemm_batch_autotune(int prec, int64_t count, const mpgemm_problem* probs, hipStream_t st,
                          int* best) {
    if (prec < 2 || prec > 4) return -1;
    if (count <= 0) return -2;
    if (!probs) return -3;
    int64_t mm = 0, nn = 0, kk = 0;
    for (int64_t q = 0; q < count; ++q) { mm += probs[q].m; nn += probs[q].n; kk += probs[q].k; }
    mm = std::max<int64_t>(1, mm / count);
    nn = std::max<int64_t>(1, nn / count);
    kk = std::max<int64_t>(1, kk / count);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MPGEMM_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return MPGEMM_ERR_HIP; }
    int chosen = -1, rc = 0;
    float best_ms = 1e30f;
    for (int c = 0; c < kPlainConfigs && !rc; ++c) {
        mpgemm_opts o{};
        o.tile = c;
        mpgemm_batch_plan* plan = nullptr;
        rc = mpgemm_batch_plan_create(prec, count, probs, &o, st, &plan);
        if (rc) break;
        rc = mpgemm_batch_plan_run(plan, st);     // warm-up
        float bms = 1e30f;
        for (int rep = 0; rep < 3 && !rc; ++rep) {
            (void)hipEventRecord(e0, st);
            rc = mpgemm_batch_plan_run(plan, st);
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) rc = MPGEMM_ERR_HIP;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            bms = std::min(bms, ms);
        }
        mpgemm_batch_plan_destroy(plan);
        if (!rc && bms < best_ms) { best_ms = bms; chosen = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        ensure_table_locked();
        g_tune[std::make_tuple(prec, 3, ilog2(mm), ilog2(nn), ilog2(kk))] = chosen;
    }
    if (best) *best = chosen;
    return 0;
}

int mpgemm_autotune_save(const char* path) {
    if (!path) return -1;
    FILE* f = std::fopen(path, "w");
    if (!f) return MPGEMM_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_table_locked();
    std::fprintf(f, "%s: prec form log2m log2n log2k tile config-list-signature\n", kTableHeader);
    for (const auto& kv : g_tune) {
        const int P = std::get<0>(kv.first), form = std::get<1>(kv.first);
        std::fprintf(f, "%d %d %d %d %d %d %08x\n", P, form, std::get<2>(kv.first), std::get<3>(kv.first),
                     std::get<4>(kv.first), kv.second, config_signature(P, form));
    }
    std::fclose(f);
    return 0;
}

int mpgemm_autotune_load(const char* path) {
    if (!path) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    ensure_table_locked();
    return load_table_locked(path);
}

// ---- slice-count rule -------------------------------------------------------

int mpgemm_tune_slices(int prec, char ta, char tb, int64_t m, int64_t n, int64_t k, const double* A,
                       int64_t lda, int64_t sa, const double* B, int64_t ldb, int64_t sb,
                       double target, int smin, int smax, hipStream_t st, int* s_out,
                       double* ratio_out) {
    // arguments: 1 prec, 2 transa, 3 transb, 4 m, 5 n, 6 k, 7 A, 8 lda, 9 a_plane_stride,
    // 10 B, 11 ldb, 12 b_plane_stride, 13 target, 14 smin, 15 smax, 16 stream, 17 s_out
    if (prec < 2 || prec > 4) return -1;
    if (!valid_trans(ta)) return -2;
    if (!valid_trans(tb)) return -3;
    if (m < 0) return -4;
    if (n < 0) return -5;
    if (k < 0) return -6;
    const int P = prec;
    const int64_t nrowa = is_trans(ta) ? k : m, ncola = is_trans(ta) ? m : k;
    const int64_t nrowb = is_trans(tb) ? n : k, ncolb = is_trans(tb) ? k : n;
    const bool reads = m > 0 && n > 0 && k > 0;
    if (reads && !A) return -7;
    if (lda < std::max<int64_t>(1, nrowa)) return -8;
    if (sa < lda * ncola) return -9;
    if (reads && !B) return -10;
    if (ldb < std::max<int64_t>(1, nrowb)) return -11;
    if (sb < ldb * ncolb) return -12;
    if (!(target > 0.0)) return -13;
    if (smin < 1 || smin > kMaxSlices) return -14;
    if (smax < smin || smax > kMaxSlices) return -15;
    if (!s_out) return -17;
    GemmArgs g{};
    g.m = m; g.n = n; g.k = k;
    g.A = A; g.lda = lda; g.sa = sa;
    g.B = B; g.ldb = ldb; g.sb = sb;
    g.ta = is_trans(ta) ? 1 : 0;
    g.tb = is_trans(tb) ? 1 : 0;
    g.alpha[0] = 1.0;
    const int64_t R = std::min<int64_t>(m, 64);
    const int64_t r0 = (m - R) / 2;
    int rc;
    if (m == 0 || n == 0 || k == 0) { *s_out = smin; if (ratio_out) *ratio_out = 0.0; return 0; }
    if (!split_k_ok(k, smax)) return MPGEMM_ERR_UNSUPPORTED;
    // the R x n sub-problem on rows r0.. of op(A)
    GemmArgs sub = g;
    sub.m = R;
    sub.A = g.ta ? g.A + r0 * g.lda : g.A + r0;
    sub.ldc = R;
    sub.sc = R * n;
    double *Cr = nullptr, *Cs = nullptr, *absab = nullptr, *ratio = nullptr;
    void* ws = nullptr;
    const size_t wsb = split_workspace_bytes(P, R, n, k, smax, 1);
    rc = 0;
    if (hipMalloc((void**)&Cr, 8 * (size_t)P * R * n) != hipSuccess ||
        hipMalloc((void**)&Cs, 8 * (size_t)P * R * n) != hipSuccess ||
        hipMalloc((void**)&absab, 8 * (size_t)R * n) != hipSuccess ||
        hipMalloc((void**)&ratio, 8 * (size_t)R * n) != hipSuccess || hipMalloc(&ws, wsb) != hipSuccess)
        rc = MPGEMM_ERR_NOMEM;
    std::vector<double> host((size_t)R * n);
    const double u = P == 2 ? std::ldexp(1.0, -104) : (P == 3 ? std::ldexp(1.0, -150) : std::ldexp(1.0, -200));
    int chosen = smax;
    double chosen_ratio = -1.0;
    if (!rc) {
        GemmArgs gr = sub;
        gr.C = Cr;
        rc = launch_plain(P, plain_default_config(P, R, n, k), gr, st) ? MPGEMM_ERR_HIP : 0;
        if (!rc) rc = launch_absdot(sub, absab, st) ? MPGEMM_ERR_HIP : 0;
    }
    for (int s = smin; s <= smax && !rc; ++s) {
        GemmArgs gs2 = sub;
        gs2.C = Cs;
        rc = launch_split(P, s, 1, gs2, ws, wsb, st) ? MPGEMM_ERR_HIP : 0;
        if (!rc)
            rc = launch_diff_ratio(P, R, n, Cs, Cr, R, R * n, absab, 1.0 / ((double)k * u), ratio, st)
                     ? MPGEMM_ERR_HIP : 0;
        if (!rc && (hipMemcpyAsync(host.data(), ratio, 8 * host.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess))
            rc = MPGEMM_ERR_HIP;
        if (rc) break;
        double mx = 0.0;
        for (double v : host) mx = std::max(mx, v);
        if (mx <= target) { chosen = s; chosen_ratio = mx; break; }
        chosen_ratio = mx;
    }
    if (Cr) (void)hipFree(Cr);
    if (Cs) (void)hipFree(Cs);
    if (absab) (void)hipFree(absab);
    if (ratio) (void)hipFree(ratio);
    if (ws) (void)hipFree(ws);
    if (rc) return rc;
    *s_out = chosen;
    if (ratio_out) *ratio_out = chosen_ratio;
    return 0;
}

// ---- misc -------------------------------------------------------------------

const char* mpgemm_strerror(int code) {
    if (code == 0) return "success";
    if (code < 0) return "invalid argument (the code is minus its 1-based position)";
    switch (code) {
    case MPGEMM_ERR_HIP: return "HIP runtime call or kernel launch failed";
    case MPGEMM_ERR_WORKSPACE: return "split form: workspace missing, misaligned or too small";
    case MPGEMM_ERR_UNSUPPORTED: return "shape or option not supported by this form";
    case MPGEMM_ERR_GRAPH: return "hipGraph capture or instantiation failed";
    case MPGEMM_ERR_ALIAS: return "C overlaps A or B";
    case MPGEMM_ERR_NOMEM: return "allocation failed";
    case MPGEMM_ERR_SCRATCH:
        return "the call needs more scratch than the library's static buffer holds "
               "(MPGEMM_STATIC_SCRATCH_BYTES)";
    default: return "unknown error";
    }
}

const char* mpgemm_version(void) { return "mpgemm 0.1.0 gfx950"; }

void mpgemm_finalize(void) {
    release_grouped_plans();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_loaded = false;          // a later use looks for the table again
}

int mpgemm_probe_peak(int which, hipStream_t st, double* rate) {
    if (which < 0 || which > 4) return -1;
    if (!rate) return -3;
    // 4096 workgroups (16 per CU); iterations sized for a few milliseconds;
    // the copy moves 1 GiB each way
    const int blocks = 4096;
    const int iters = which == 3 ? 4096 : 16384;
    const int64_t copy_n = (int64_t)1 << 27;
    const size_t out_elems = which == 4 ? (size_t)2 * copy_n : (size_t)blocks * 256;
    double* out = nullptr;
    if (hipMalloc((void**)&out, sizeof(double) * out_elems) != hipSuccess) return MPGEMM_ERR_NOMEM;
    hipEvent_t e0, e1;
    int rc = 0;
    if (hipEventCreate(&e0) != hipSuccess) rc = MPGEMM_ERR_HIP;
    if (!rc && hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); rc = MPGEMM_ERR_HIP; }
    double ops = 0.0;
    float best = 1e30f;
    if (!rc) {
        for (int rep = 0; rep < 4 && !rc; ++rep) {      // first run warms up
            (void)hipEventRecord(e0, st);
            rc = (which == 4 ? launch_probe_copy(out, out + copy_n, copy_n, &ops, st)
                             : launch_probe(which, out, blocks, iters, &ops, st))
                     ? MPGEMM_ERR_HIP
                     : 0;
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) rc = MPGEMM_ERR_HIP;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) best = std::min(best, ms);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    (void)hipFree(out);
    if (rc) return rc;
    *rate = ops / (best * 1e-3);
    return 0;
}

}  // extern "C"
