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
// bitwise that of the same recursion evaluated on the CPU.
//
// The recursion runs breadth first, which suits the GPU: level l has 7^l
// nodes of size m/2^l x n/2^l x k/2^l.  A down-sweep forms the operands of
// all nodes of a level (one launch per formula, batched over the parents);
// all 7^L leaf products then run as one strided batch of the plain kernel
// (enough tiles to fill the chip even when a leaf alone would not); an
// up-sweep combines the seven results of every parent, level by level.  Each
// value is produced by exactly the operations of the depth-first recursion,
// in the same order.  Block sums are HBM-bound element-wise passes.  All
// temporaries live in the caller's workspace, dense column-major, node after
// node: the product R_0 (m x n), then per level l = 1..L the operands of A
// and B and the results R_l of its nodes.
#pragma clang fp contract(off)

#include "internal.hpp"
#include "mp_arith.hpp"

namespace mpg {

// The seven products: operand of A (and of B) for child i is quadrant q1, or
// q1 + q2, or q1 - q2 of the parent's operand.
struct Term {
    int q1i, q1j, q2i, q2j, mode;     // mode 0: copy q1; 1: q1 + q2; 2: q1 - q2
};
static const Term kA[7] = {{0, 0, 1, 1, 1}, {1, 0, 1, 1, 1}, {0, 0, 0, 0, 0}, {1, 1, 1, 1, 0},
                           {0, 0, 0, 1, 1}, {1, 0, 0, 0, 2}, {0, 1, 1, 1, 2}};
static const Term kB[7] = {{0, 0, 1, 1, 1}, {0, 0, 0, 0, 0}, {0, 1, 1, 1, 2}, {1, 0, 0, 0, 2},
                           {1, 1, 1, 1, 0}, {0, 0, 0, 1, 1}, {1, 0, 1, 1, 1}};
// Combination of the seven results into the parent's quadrants, in order:
// {quadrant i, j; first operand: child c1, or the quadrant itself when c1 < 0;
//  second operand child c2; subtract?}
struct Comb {
    int qi, qj, c1, c2, neg;
};
static const Comb kC[8] = {{0, 0, 0, 3, 0}, {0, 0, -1, 4, 1}, {0, 0, -1, 6, 0},   // C11 = M1 + M4 - M5 + M7
                           {0, 1, 2, 4, 0},                                        // C12 = M3 + M5
                           {1, 0, 1, 3, 0},                                        // C21 = M2 + M4
                           {1, 1, 0, 1, 1}, {1, 1, -1, 2, 0}, {1, 1, -1, 5, 0}};   // C22 = M1 - M2 + M3 + M6

// Down-sweep: child `child` of every parent p = blockIdx.y: an h x w block
// (h x w is the child's size) formed from quadrants of the parent's operand
// (element (r, c) of component q at src + p snode + q sps + (t ? c + r sld :
// r + c sld)); written dense at dst + (7 p + child) dnode.
template <int P>
__global__ __launch_bounds__(256) void bfs_down_kernel(int64_t h, int64_t w, const double* __restrict__ src,
                                                       int64_t sld, int64_t sps, int st, int64_t snode, Term tm,
                                                       double* __restrict__ dst, int64_t dnode, int child) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * w) return;
    const int64_t i = idx % h, j = idx / h;
    const int64_t p = blockIdx.y;
    const double* base = src + p * snode;
    auto at = [&](int qi, int qj) -> int64_t {
        const int64_t r = qi * h + i, c = qj * w + j;
        return st ? c + r * sld : r + c * sld;
    };
    const int64_t o1 = at(tm.q1i, tm.q1j);
    mp<P> x;
#pragma unroll
    for (int q = 0; q < P; ++q) x.c[q] = base[q * sps + o1];
    if (tm.mode != 0) {
        const int64_t o2 = at(tm.q2i, tm.q2j);
        mp<P> y;
#pragma unroll
        for (int q = 0; q < P; ++q) y.c[q] = tm.mode == 2 ? -base[q * sps + o2] : base[q * sps + o2];
        x = add(x, y);
    }
    double* out = dst + (7 * p + child) * dnode;
#pragma unroll
    for (int q = 0; q < P; ++q) out[q * h * w + i + j * h] = x.c[q];
}

// Up-sweep: one combination step for every parent p = blockIdx.y.  Children
// results are dense h x w at R + (7 p + c) rnode; the parent is dense 2h x 2w
// at out + p onode (leading dimension 2h, plane stride 4hw).
template <int P>
__global__ __launch_bounds__(256) void bfs_up_kernel(int64_t h, int64_t w, const double* __restrict__ R,
                                                     int64_t rnode, Comb cb, double* __restrict__ out,
                                                     int64_t onode) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * w) return;
    const int64_t i = idx % h, j = idx / h;
    const int64_t p = blockIdx.y;
    double* par = out + p * onode;
    const int64_t pps = 4 * h * w;
    const int64_t po = (cb.qi * h + i) + (cb.qj * w + j) * (2 * h);
    mp<P> x, y;
    if (cb.c1 < 0) {
#pragma unroll
        for (int q = 0; q < P; ++q) x.c[q] = par[q * pps + po];
    } else {
        const double* r1 = R + (7 * p + cb.c1) * rnode;
#pragma unroll
        for (int q = 0; q < P; ++q) x.c[q] = r1[q * h * w + i + j * h];
    }
    const double* r2 = R + (7 * p + cb.c2) * rnode;
#pragma unroll
    for (int q = 0; q < P; ++q) y.c[q] = cb.neg ? -r2[q * h * w + i + j * h] : r2[q * h * w + i + j * h];
    const mp<P> r = add(x, y);
#pragma unroll
    for (int q = 0; q < P; ++q) par[q * pps + po] = r.c[q];
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

static int64_t pow7(int l) {
    int64_t r = 1;
    for (int i = 0; i < l; ++i) r *= 7;
    return r;
}

// Workspace doubles: R_0 plus, per level, operands and results of its nodes.
size_t strassen_workspace_bytes(int P, int levels, int64_t m, int64_t n, int64_t k) {
    size_t d = (size_t)P * m * n;
    for (int l = 1; l <= levels; ++l) {
        const int64_t h = m >> l, w = n >> l, q = k >> l;
        d += (size_t)pow7(l) * P * (h * q + q * w + h * w);
    }
    return d * 8;
}

template <int P>
static void down(int64_t h, int64_t w, const double* src, int64_t sld, int64_t sps, int st, int64_t snode,
                 int64_t parents, const Term& t, double* dst, int64_t dnode, int child, hipStream_t s) {
    const dim3 gr((unsigned)((h * w + 255) / 256), (unsigned)parents), bl(256);
    hipLaunchKernelGGL(bfs_down_kernel<P>, gr, bl, 0, s, h, w, src, sld, sps, st, snode, t, dst, dnode, child);
}

template <int P>
static void up(int64_t h, int64_t w, const double* R, int64_t rnode, const Comb& c, double* out,
               int64_t onode, int64_t parents, hipStream_t s) {
    const dim3 gr((unsigned)((h * w + 255) / 256), (unsigned)parents), bl(256);
    hipLaunchKernelGGL(bfs_up_kernel<P>, gr, bl, 0, s, h, w, R, rnode, c, out, onode);
}

template <int P>
static int strassen_bfs(int levels, const GemmArgs& g, double* ws, hipStream_t st,
                        int (*pick)(int, int64_t, int64_t, int64_t)) {
    // workspace sections
    double* R[8];
    double* XA[8];
    double* YB[8];
    double* cur = ws;
    R[0] = cur;
    cur += (int64_t)P * g.m * g.n;
    for (int l = 1; l <= levels; ++l) {
        const int64_t N = pow7(l), h = g.m >> l, w = g.n >> l, q = g.k >> l;
        XA[l] = cur; cur += N * P * h * q;
        YB[l] = cur; cur += N * P * q * w;
        R[l] = cur;  cur += N * P * h * w;
    }
    // down-sweep
    for (int l = 1; l <= levels; ++l) {
        const int64_t parents = pow7(l - 1);
        const int64_t h = g.m >> l, w = g.n >> l, q = g.k >> l;
        const int64_t ph = h * 2, pw = w * 2, pq = q * 2;     // parent sizes
        const double* sa = l == 1 ? g.A : XA[l - 1];
        const double* sb = l == 1 ? g.B : YB[l - 1];
        const int64_t a_ld = l == 1 ? g.lda : ph, a_ps = l == 1 ? g.sa : ph * pq;
        const int64_t b_ld = l == 1 ? g.ldb : pq, b_ps = l == 1 ? g.sb : pq * pw;
        const int a_t = l == 1 ? g.ta : 0, b_t = l == 1 ? g.tb : 0;
        const int64_t a_node = (int64_t)P * ph * pq, b_node = (int64_t)P * pq * pw;
        for (int c = 0; c < 7; ++c) {
            down<P>(h, q, sa, a_ld, a_ps, a_t, a_node, parents, kA[c], XA[l], (int64_t)P * h * q, c, st);
            down<P>(q, w, sb, b_ld, b_ps, b_t, b_node, parents, kB[c], YB[l], (int64_t)P * q * w, c, st);
        }
    }
    int rc = (int)hipGetLastError();
    if (rc) return rc;
    // the 7^L leaf products, one launch
    {
        const int64_t h = g.m >> levels, w = g.n >> levels, q = g.k >> levels;
        GemmArgs lg{};
        lg.m = h; lg.n = w; lg.k = q;
        lg.A = XA[levels]; lg.lda = h; lg.sa = h * q;
        lg.B = YB[levels]; lg.ldb = q; lg.sb = q * w;
        lg.C = R[levels]; lg.ldc = h; lg.sc = h * w;
        lg.alpha[0] = 1.0;
        // the batch as a whole is as parallel as the full product: tile for that
        rc = launch_plain_strided(P, pick(P, g.m, g.n, q), lg, pow7(levels), (int64_t)P * h * q,
                                  (int64_t)P * q * w, (int64_t)P * h * w, st);
        if (rc) return rc;
    }
    // up-sweep
    for (int l = levels; l >= 1; --l) {
        const int64_t parents = pow7(l - 1);
        const int64_t h = g.m >> l, w = g.n >> l;
        for (int c = 0; c < 8; ++c)
            up<P>(h, w, R[l], (int64_t)P * h * w, kC[c], R[l - 1], (int64_t)P * 4 * h * w, parents, st);
    }
    rc = (int)hipGetLastError();
    if (rc) return rc;
    const int64_t blocks = (g.m * g.n + 255) / 256;
    hipLaunchKernelGGL(strassen_epilogue_kernel<P>, dim3((unsigned)blocks), dim3(256), 0, st, g,
                       (const double*)R[0]);
    return (int)hipGetLastError();
}

// Caller: arguments validated, m, n, k > 0 divisible by 2^levels
// (1 <= levels <= 5), alpha != 0, workspace of strassen_workspace_bytes().
int launch_strassen(int P, int levels, const GemmArgs& g, void* ws, hipStream_t st,
                    int (*pick)(int, int64_t, int64_t, int64_t)) {
    if (levels < 1 || levels > 5) return (int)hipErrorInvalidValue;
    // grid limits: blocks of the largest pass and 7^(L-1) parents per launch
    const int64_t blocks = (g.m * g.n + 255) / 256;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    if (P == 2) return strassen_bfs<2>(levels, g, (double*)ws, st, pick);
    if (P == 3) return strassen_bfs<3>(levels, g, (double*)ws, st, pick);
    return strassen_bfs<4>(levels, g, (double*)ws, st, pick);
}

}  // namespace mpg
