// strassen.hip -- Strassen's method over the plain GEMM (Sec. 3, Fig. 5).
//
// For m, n, k divisible by 2^L, op(A), op(B) and the product are cut into
// 2 x 2 blocks and the product is formed from seven block products, for L
// levels; the blocks at the bottom go through the plain kernel (canonical
// order, alpha = 1, beta = 0).  The scheme is Strassen's original one:
//   M1 = (A11 + A22)(B11 + B22)   M2 = (A21 + A22) B11
//   M3 = A11 (B12 - B22)          M4 = A22 (B21 - B11)
//   M5 = (A11 + A12) B22          M6 = (A21 - A11)(B11 + B12)
//   M7 = (A12 - A22)(B21 + B22)
//   C11 = M1 + M4 - M5 + M7       C12 = M3 + M5
//   C21 = M2 + M4                 C22 = M1 - M2 + M3 + M6
// with sums left to right and x - y = ADD(x, -y) (exact negation).  The
// product then goes through the plain form's epilogue, so the result is
// bitwise that of the same recursion evaluated on the CPU.  Block sums are
// HBM-bound element-wise kernels; the block products are the plain kernel at
// a quarter (per level) of the size.  All temporaries live in the caller's
// workspace: the product (m x n), then per level the two operand sums and the
// seven block products; the seven recursive calls of a level run one after
// another on the stream and share the deeper levels' region.
#pragma clang fp contract(off)

#include "internal.hpp"
#include "mp_arith.hpp"

namespace mpg {

// Dense view in op space: element (i, j), component c at
// p[c * ps + (t ? j + i * ld : i + j * ld)].
struct MView {
    double* p;
    int64_t ld, ps;
    int t;
};

static MView block(MView v, int bi, int bj, int64_t h, int64_t w) {
    MView r = v;
    r.p = v.t ? v.p + bj * w + (int64_t)bi * h * v.ld : v.p + bi * h + (int64_t)bj * w * v.ld;
    return r;
}

template <int P>
__device__ __forceinline__ mp<P> view_get(const MView& v, int64_t i, int64_t j) {
    const int64_t off = v.t ? j + i * v.ld : i + j * v.ld;
    mp<P> x;
#pragma unroll
    for (int c = 0; c < P; ++c) x.c[c] = v.p[c * v.ps + off];
    return x;
}

// R = X + sign Y over h x w (R is a non-transposed view); one entry per
// thread, i fastest.
template <int P>
__global__ __launch_bounds__(256) void block_addsub_kernel(int64_t h, int64_t w, MView X, MView Y,
                                                           int neg, MView R) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * w) return;
    const int64_t i = idx % h, j = idx / h;
    const mp<P> x = view_get<P>(X, i, j);
    mp<P> y = view_get<P>(Y, i, j);
    if (neg) {
#pragma unroll
        for (int c = 0; c < P; ++c) y.c[c] = -y.c[c];
    }
    const mp<P> r = add(x, y);
#pragma unroll
    for (int c = 0; c < P; ++c) R.p[c * R.ps + i + j * R.ld] = r.c[c];
}

// C = alpha PR + beta C (C not read when beta == 0), the plain epilogue.
template <int P>
__global__ __launch_bounds__(256) void strassen_epilogue_kernel(GemmArgs g, const double* __restrict__ PR) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.m * g.n) return;
    const int64_t i = idx % g.m, j = idx / g.m;
    mp<P> alpha, beta, acc;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        alpha.c[c] = g.alpha[c];
        beta.c[c] = g.beta[c];
        acc.c[c] = PR[c * g.m * g.n + idx];
    }
    const int64_t off = i + j * g.ldc;
    mp<P> t = mul(alpha, acc);
    if (!mp_is_zero(beta)) {
        mp<P> co;
#pragma unroll
        for (int c = 0; c < P; ++c) co.c[c] = g.C[c * g.sc + off];
        t = add(t, mul(beta, co));
    }
#pragma unroll
    for (int c = 0; c < P; ++c) g.C[c * g.sc + off] = t.c[c];
}

static int launch_addsub(int P, int64_t h, int64_t w, const MView& X, const MView& Y, int neg,
                         const MView& R, hipStream_t st) {
    const int64_t blocks = (h * w + 255) / 256;
    if (blocks <= 0) return 0;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    const dim3 gr((unsigned)blocks), bl(256);
    if (P == 2) hipLaunchKernelGGL(block_addsub_kernel<2>, gr, bl, 0, st, h, w, X, Y, neg, R);
    else if (P == 3) hipLaunchKernelGGL(block_addsub_kernel<3>, gr, bl, 0, st, h, w, X, Y, neg, R);
    else hipLaunchKernelGGL(block_addsub_kernel<4>, gr, bl, 0, st, h, w, X, Y, neg, R);
    return (int)hipGetLastError();
}

// Doubles of workspace below one level of the recursion for an h x w
// product with inner dimension q (its own temporaries plus the deeper ones).
static int64_t level_doubles(int P, int levels, int64_t h, int64_t w, int64_t q) {
    if (levels == 0) return 0;
    const int64_t a = h / 2, b = w / 2, c = q / 2;
    return (int64_t)P * (a * c + c * b + 7 * a * b) + level_doubles(P, levels - 1, a, b, c);
}

size_t strassen_workspace_bytes(int P, int levels, int64_t m, int64_t n, int64_t k) {
    return (size_t)8 * ((size_t)P * m * n + (size_t)level_doubles(P, levels, m, n, k));
}

static MView dense(double* p, int64_t h, int64_t w) { return MView{p, h > 0 ? h : 1, h * w, 0}; }

// Out (h x w) = X (h x q) Y (q x w) with `levels` levels; ws holds
// level_doubles(...) doubles.
static int strassen_rec(int P, int levels, int64_t h, int64_t w, int64_t q, const MView& X,
                        const MView& Y, const MView& Out, double* ws, hipStream_t st,
                        int (*pick)(int, int64_t, int64_t, int64_t)) {
    if (levels == 0) {
        GemmArgs g{};
        g.ta = X.t;
        g.tb = Y.t;
        g.m = h; g.n = w; g.k = q;
        g.A = X.p; g.lda = X.ld; g.sa = X.ps;
        g.B = Y.p; g.ldb = Y.ld; g.sb = Y.ps;
        g.C = Out.p; g.ldc = Out.ld; g.sc = Out.ps;
        g.alpha[0] = 1.0;
        return launch_plain(P, pick(P, h, w, q), g, st);
    }
    const int64_t a = h / 2, b = w / 2, c = q / 2;
    const MView A11 = block(X, 0, 0, a, c), A12 = block(X, 0, 1, a, c);
    const MView A21 = block(X, 1, 0, a, c), A22 = block(X, 1, 1, a, c);
    const MView B11 = block(Y, 0, 0, c, b), B12 = block(Y, 0, 1, c, b);
    const MView B21 = block(Y, 1, 0, c, b), B22 = block(Y, 1, 1, c, b);
    const MView C11 = block(Out, 0, 0, a, b), C12 = block(Out, 0, 1, a, b);
    const MView C21 = block(Out, 1, 0, a, b), C22 = block(Out, 1, 1, a, b);
    double* cur = ws;
    const MView SA = dense(cur, a, c); cur += (int64_t)P * a * c;
    const MView SB = dense(cur, c, b); cur += (int64_t)P * c * b;
    MView M[7];
    for (int i = 0; i < 7; ++i) { M[i] = dense(cur, a, b); cur += (int64_t)P * a * b; }
    double* deeper = cur;
    int rc = 0;
#define MPG_TRY(x) if (!rc) rc = (x)
    MPG_TRY(launch_addsub(P, a, c, A11, A22, 0, SA, st));
    MPG_TRY(launch_addsub(P, c, b, B11, B22, 0, SB, st));
    MPG_TRY(strassen_rec(P, levels - 1, a, b, c, SA, SB, M[0], deeper, st, pick));
    MPG_TRY(launch_addsub(P, a, c, A21, A22, 0, SA, st));
    MPG_TRY(strassen_rec(P, levels - 1, a, b, c, SA, B11, M[1], deeper, st, pick));
    MPG_TRY(launch_addsub(P, c, b, B12, B22, 1, SB, st));
    MPG_TRY(strassen_rec(P, levels - 1, a, b, c, A11, SB, M[2], deeper, st, pick));
    MPG_TRY(launch_addsub(P, c, b, B21, B11, 1, SB, st));
    MPG_TRY(strassen_rec(P, levels - 1, a, b, c, A22, SB, M[3], deeper, st, pick));
    MPG_TRY(launch_addsub(P, a, c, A11, A12, 0, SA, st));
    MPG_TRY(strassen_rec(P, levels - 1, a, b, c, SA, B22, M[4], deeper, st, pick));
    MPG_TRY(launch_addsub(P, a, c, A21, A11, 1, SA, st));
    MPG_TRY(launch_addsub(P, c, b, B11, B12, 0, SB, st));
    MPG_TRY(strassen_rec(P, levels - 1, a, b, c, SA, SB, M[5], deeper, st, pick));
    MPG_TRY(launch_addsub(P, a, c, A12, A22, 1, SA, st));
    MPG_TRY(launch_addsub(P, c, b, B21, B22, 0, SB, st));
    MPG_TRY(strassen_rec(P, levels - 1, a, b, c, SA, SB, M[6], deeper, st, pick));
    // C11 = M1 + M4 - M5 + M7, C12 = M3 + M5, C21 = M2 + M4, C22 = M1 - M2 + M3 + M6
    MPG_TRY(launch_addsub(P, a, b, M[0], M[3], 0, C11, st));
    MPG_TRY(launch_addsub(P, a, b, C11, M[4], 1, C11, st));
    MPG_TRY(launch_addsub(P, a, b, C11, M[6], 0, C11, st));
    MPG_TRY(launch_addsub(P, a, b, M[2], M[4], 0, C12, st));
    MPG_TRY(launch_addsub(P, a, b, M[1], M[3], 0, C21, st));
    MPG_TRY(launch_addsub(P, a, b, M[0], M[1], 1, C22, st));
    MPG_TRY(launch_addsub(P, a, b, C22, M[2], 0, C22, st));
    MPG_TRY(launch_addsub(P, a, b, C22, M[5], 0, C22, st));
#undef MPG_TRY
    return rc;
}

// Caller: arguments validated, m, n, k > 0 divisible by 2^levels, alpha != 0,
// workspace of strassen_workspace_bytes() at ws.
int launch_strassen(int P, int levels, const GemmArgs& g, void* ws, hipStream_t st,
                    int (*pick)(int, int64_t, int64_t, int64_t)) {
    double* PR = (double*)ws;
    const MView X{const_cast<double*>(g.A), g.lda, g.sa, g.ta ? 1 : 0};
    const MView Y{const_cast<double*>(g.B), g.ldb, g.sb, g.tb ? 1 : 0};
    int rc = strassen_rec(P, levels, g.m, g.n, g.k, X, Y, dense(PR, g.m, g.n),
                          PR + (int64_t)P * g.m * g.n, st, pick);
    if (rc) return rc;
    const int64_t blocks = (g.m * g.n + 255) / 256;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    const dim3 gr((unsigned)blocks), bl(256);
    if (P == 2) hipLaunchKernelGGL(strassen_epilogue_kernel<2>, gr, bl, 0, st, g, PR);
    else if (P == 3) hipLaunchKernelGGL(strassen_epilogue_kernel<3>, gr, bl, 0, st, g, PR);
    else hipLaunchKernelGGL(strassen_epilogue_kernel<4>, gr, bl, 0, st, g, PR);
    return (int)hipGetLastError();
}

}  // namespace mpg
