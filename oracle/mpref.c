/*
 * mpref.c -- plain CPU oracle for double-double (DD), triple-double (TD) and
 * quad-double (QD) matrix multiplication built from error-free transformations
 * (Kouya, "Acceleration of multiple precision matrix multiplication based on
 * multi-component floating-point arithmetic using AVX2", arXiv 2101.06584).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path links,
 * loads or calls this file; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no source with the GPU code.
 *
 * It is deliberately scalar and unblocked: one multi-component number at a
 * time, each operation in the order the paper prints it, so that a reader can
 * check it against Algorithms 1-6 by eye.  Built with -ffp-contract=off and no
 * fast-math: every '+', '-', '*' is one IEEE-754 binary64 operation in
 * round-to-nearest-even, and fma() is the correctly rounded fused multiply-add.
 *
 * Readings of points the paper leaves open (TwoSum/QuickTwoSum/TwoProd bodies,
 * ThreeSum, ThreeSum2, VecSum, VSEB(k), Renorm, the missing t3 line of the QD
 * addition, the dead first line of the QD multiplication, the TD addition
 * through the QD one, the GEMM summation order) are stated at each function.
 *
 * Parity pins: every function here is pinned by the CPU tests (exact rational
 * invariants, error bounds against the exact result, closed forms, brute
 * force on small inputs).  Parity unpinned: none.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: error-free transformations.                                    */
/* ------------------------------------------------------------------------ */

/* QuickTwoSum (Dekker's Fast2Sum): s = fl(a+b), e = b - (s - a).  Exact
 * (s + e == a + b) when exponent(a) >= exponent(b). */
static void quick_two_sum(double a, double b, double *s, double *e)
{
    double sum = a + b;
    double back = sum - a;
    *e = b - back;
    *s = sum;
}

/* TwoSum (Knuth), in the operation order spelled out lane by lane in the QD
 * addition (Algorithm 5): s, v = s - a, u = s - v, w = a - u, u' = b - v,
 * e = w + u'.  Always exact. */
static void two_sum(double a, double b, double *s, double *e)
{
    double sum = a + b;
    double v = sum - a;
    double u = sum - v;
    double w = a - u;
    double u2 = b - v;
    *e = w + u2;
    *s = sum;
}

/* TwoProd with FMA: p = fl(ab), e = fma(a, b, -p) = ab - p exactly (barring
 * underflow). */
static void two_prod(double a, double b, double *p, double *e)
{
    double prod = a * b;
    *e = fma(a, b, -prod);
    *p = prod;
}

/* ThreeSum (a, b, c) -> (a', b', c'), three TwoSums, sum preserved exactly.
 * Not printed in the paper; read as the three-term sum of the quad-double
 * algorithms the paper builds on (its QD library reference). */
static void three_sum(double *a, double *b, double *c)
{
    double t1, t2, t3;
    two_sum(*a, *b, &t1, &t2);
    two_sum(*c, t1, a, &t3);
    two_sum(t2, t3, b, c);
}

/* ThreeSum2 (a, b, c) -> (a', b'): the first two TwoSums of ThreeSum, then a
 * rounded add of the two error terms. */
static void three_sum2(double *a, double *b, double c)
{
    double t1, t2, t3;
    two_sum(*a, *b, &t1, &t2);
    two_sum(c, t1, a, &t3);
    *b = t2 + t3;
}

/* VecSum (Sec. 2.3, from the triple-word arithmetic the paper cites): a
 * bottom-up chain of TwoSums, s = x[n-1]; for i = n-2..0:
 * (s, e[i+1]) = TwoSum(x[i], s); e[0] = s.  Error-free.  x and e may alias. */
static void vec_sum(const double *x, int n, double *e)
{
    double s = x[n - 1];
    for (int i = n - 2; i >= 0; --i)
        two_sum(x[i], s, &s, &e[i + 1]);
    e[0] = s;
}

/* VSEB(k) ("VecSum with branch", Sec. 2.3): a top-down QuickTwoSum pass that
 * keeps a partial sum while the rounding error is zero and emits it as the
 * next output term otherwise; after k terms the rest is dropped.  Outputs not
 * reached are zero.  The test "error != 0" treats -0 as zero. */
static void vseb(const double *e, int n, double *r, int k)
{
    for (int q = 0; q < k; ++q)
        r[q] = 0.0;
    int j = 0;
    double carry = e[0];
    for (int i = 1; i < n; ++i) {
        double s, t;
        quick_two_sum(carry, e[i], &s, &t);
        if (t != 0.0) {
            r[j++] = s;
            carry = t;
            if (j == k)
                return;
        } else {
            carry = s;
        }
    }
    r[j] = carry;
}

/* Renorm (the renormalisation Sec. 2 asks to be written as plain loops, so
 * that it vectorises): five terms to a
 * four-component number.
 * Pass 1: bottom-up QuickTwoSum chain c4 -> c0 giving e[0..4].
 * Pass 2: top-down, the pair (e0, e1) as produced by pass 1, then
 * QuickTwoSum(carry, e[i]) for i = 2..4; a non-zero error term closes an
 * output slot (the sum becomes that slot, the error the new carry).  When the
 * third slot closes, the last slot takes the carry plus the remaining e's
 * (plain adds, left to right).  Otherwise the carry fills the next open slot
 * and later slots are zero. */
static void renorm4(double c0, double c1, double c2, double c3, double c4, double r[4])
{
    double e[5];
    double s;
    quick_two_sum(c3, c4, &s, &e[4]);
    quick_two_sum(c2, s, &s, &e[3]);
    quick_two_sum(c1, s, &s, &e[2]);
    quick_two_sum(c0, s, &s, &e[1]);
    e[0] = s;

    r[0] = r[1] = r[2] = r[3] = 0.0;
    int j = 0;
    double carry = 0.0;
    for (int i = 1; i <= 4; ++i) {
        double sv, t;
        if (i == 1) {
            sv = e[0];
            t = e[1];
        } else {
            quick_two_sum(carry, e[i], &sv, &t);
        }
        if (t != 0.0) {
            r[j++] = sv;
            carry = t;
            if (j == 3) {
                double tail = carry;
                for (int q = i + 1; q <= 4; ++q)
                    tail = tail + e[q];
                r[3] = tail;
                return;
            }
        } else {
            carry = sv;
        }
    }
    r[j] = carry;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2: DD addition (Algorithm 1) and multiplication (Algorithm 2).    */
/* ------------------------------------------------------------------------ */

static void dd_add(const double *x, const double *y, double *r)
{
    double s, e;
    two_sum(x[0], y[0], &s, &e);
    double w = x[1] + y[1];
    e = e + w;
    quick_two_sum(s, e, &r[0], &r[1]);
}

/* Algorithm 2: the two cross products are separate rounded multiplies and
 * the sums separate rounded adds (no fused multiply-add there). */
static void dd_mul(const double *x, const double *y, double *r)
{
    double p1, p2;
    two_prod(x[0], y[0], &p1, &p2);
    double w1 = x[0] * y[1];
    double w2 = x[1] * y[0];
    double w3 = w1 + w2;
    p2 = p2 + w3;
    quick_two_sum(p1, p2, &r[0], &r[1]);
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.4: QD addition (Algorithm 5) and multiplication (Algorithm 6).    */
/* ------------------------------------------------------------------------ */

/* QD addition.  Each component pair x_i + y_i is added exactly (TwoSum: sum
 * s_i, error t_i).  The errors are then carried one level down: level 1 takes
 * t_0 (one carry out), level 2 that carry and t_1 (ThreeSum, two carries
 * out), level 3 the first of them and t_2 (ThreeSum2, one carry out); the
 * fifth term is the two remaining carries plus t_3, and Renorm makes four
 * components of the five terms.  The algorithm's tail uses a fourth error
 * term that its text never defines; read as t_3, the error of the fourth
 * pair's TwoSum, like the other three. */
static void qd_add(const double *x, const double *y, double *r)
{
    double s[4], t[4];
    for (int i = 0; i < 4; ++i)
        two_sum(x[i], y[i], &s[i], &t[i]);
    double carry = t[0], carry2 = t[1];
    two_sum(s[1], carry, &s[1], &carry);
    three_sum(&s[2], &carry, &carry2);
    three_sum2(&s[3], &carry, t[2]);
    double tail = (carry + carry2) + t[3];
    renorm4(s[0], s[1], s[2], s[3], tail, r);
}

/* QD multiplication.  The component products x_i y_j of order eps^0 to
 * eps^2 (i + j <= 2) are split exactly by TwoProd into p_ij + q_ij.  Order
 * eps: ThreeSum of p01, p10 and q00.  Order eps^2: that sum's first carry
 * with q01 and q10 (ThreeSum), and p02 + p11 + p20 (ThreeSum); the two are
 * combined by TwoSums into the order-eps^2 component and a lower term.  The
 * order-eps^3 rest is added in rounded arithmetic, one term at a time in the
 * paper's order: x0 y3, x1 y2, x2 y1, x3 y0, then the errors q00, q02, q11,
 * q20.  Renorm makes four components of the five terms.  A sum of the
 * leading components that the algorithm computes first is overwritten
 * before any use; it is left out. */
static void qd_mul(const double *x, const double *y, double *r)
{
    double p00, q00, p01, q01, p10, q10, p02, q02, p11, q11, p20, q20;
    two_prod(x[0], y[0], &p00, &q00);
    two_prod(x[0], y[1], &p01, &q01);
    two_prod(x[1], y[0], &p10, &q10);
    two_prod(x[0], y[2], &p02, &q02);
    two_prod(x[1], y[1], &p11, &q11);
    two_prod(x[2], y[0], &p20, &q20);

    three_sum(&p01, &p10, &q00);
    three_sum(&p10, &q01, &q10);
    three_sum(&p02, &p11, &p20);

    double hi, hi_err, mid, mid_err;
    two_sum(p10, p02, &hi, &hi_err);
    two_sum(q01, p11, &mid, &mid_err);
    double lo = q10 + p20;
    two_sum(mid, hi_err, &mid, &hi_err);
    lo = lo + (hi_err + mid_err);

    for (int i = 0; i < 4; ++i)
        mid = mid + x[i] * y[3 - i];
    const double errs[4] = {q00, q02, q11, q20};
    for (int i = 0; i < 4; ++i)
        mid = mid + errs[i];
    renorm4(p00, p01, hi, mid, lo, r);
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.3: TD addition (TDaddq) and multiplication (Algorithm 4).         */
/* ------------------------------------------------------------------------ */

/* TDaddq: the QD addition applied to (x0, x1, x2, 0) and (y0, y1, y2, 0), the
 * paper's default TD addition; the fourth output component is dropped. */
static void td_addq(const double *x, const double *y, double *r)
{
    double xq[4] = {x[0], x[1], x[2], 0.0};
    double yq[4] = {y[0], y[1], y[2], 0.0};
    double rq[4];
    qd_add(xq, yq, rq);
    r[0] = rq[0];
    r[1] = rq[1];
    r[2] = rq[2];
}

/* Algorithm 4 ("fast" triple-word product).  b0..b2 are VecSum outputs, not
 * operand components. */
static void td_mul(const double *x, const double *y, double *r)
{
    double z00u, z00l, z01u, z01l, z10u, z10l;
    two_prod(x[0], y[0], &z00u, &z00l);
    two_prod(x[0], y[1], &z01u, &z01l);
    two_prod(x[1], y[0], &z10u, &z10l);
    double in3[3] = {z00l, z01u, z10u};
    double b[3];
    vec_sum(in3, 3, b);
    double c = fma(x[1], y[1], b[2]);
    double z31 = fma(x[0], y[2], z10l);
    double z32 = fma(x[2], y[0], z01l);
    double z3 = z31 + z32;
    double s3 = c + z3;
    double in4[4] = {z00u, b[0], b[1], s3};
    double e[4];
    vec_sum(in4, 4, e);
    r[0] = e[0];
    vseb(&e[1], 3, &r[1], 2);
}

/* The other TD operations of Sec. 2.3, which the paper measures but does not
 * adopt for its TD matrix multiplication.
 *
 * Merge (first step of Algorithm 3): the six components of x and y in order
 * of decreasing magnitude, by the two-pointer merge of the two expansions:
 * take the head of x when its magnitude is at least that of y's head,
 * otherwise y's head.  On normalised operands (each ordered by decreasing
 * magnitude) this is the stable sort of (x0, x1, x2, y0, y1, y2) by
 * decreasing |.|, x before y on equal magnitudes. */
static void merge_mag(const double *x, int nx, const double *y, int ny, double *z)
{
    int i = 0, j = 0;
    for (int k = 0; k < nx + ny; ++k) {
        if (j >= ny || (i < nx && fabs(x[i]) >= fabs(y[j])))
            z[k] = x[i++];
        else
            z[k] = y[j++];
    }
}

/* Algorithm 3 (the accurate TD addition, TDadd): Merge, VecSum over the six
 * terms, VSEB(3). */
static void td_add_acc(const double *x, const double *y, double *r)
{
    double z[6], e[6];
    merge_mag(x, 3, y, 3, z);
    vec_sum(z, 6, e);
    vseb(e, 6, r, 3);
}

/* TDmulq: the QD multiplication applied to (x0, x1, x2, 0) and (y0, y1, y2, 0),
 * fourth output dropped (the TD product "converted to QDmul" that the paper
 * tried). */
static void td_mulq(const double *x, const double *y, double *r)
{
    double xq[4] = {x[0], x[1], x[2], 0.0};
    double yq[4] = {y[0], y[1], y[2], 0.0};
    double rq[4];
    qd_mul(xq, yq, rq);
    r[0] = rq[0];
    r[1] = rq[1];
    r[2] = rq[2];
}

/* ------------------------------------------------------------------------ */
/* Precision dispatch.  `variant` selects the TD operations (P == 3 only):  */
/* bit 0 the accurate addition (Algorithm 3) instead of TDaddq, bit 1       */
/* TDmulq instead of Algorithm 4.                                           */
/* ------------------------------------------------------------------------ */

static void mp_add_v(int P, int variant, const double *x, const double *y, double *r)
{
    if (P == 2)
        dd_add(x, y, r);
    else if (P == 3)
        (variant & 1) ? td_add_acc(x, y, r) : td_addq(x, y, r);
    else
        qd_add(x, y, r);
}

static void mp_mul_v(int P, int variant, const double *x, const double *y, double *r)
{
    if (P == 2)
        dd_mul(x, y, r);
    else if (P == 3)
        (variant & 2) ? td_mulq(x, y, r) : td_mul(x, y, r);
    else
        qd_mul(x, y, r);
}

static void mp_add(int P, const double *x, const double *y, double *r) { mp_add_v(P, 0, x, y, r); }
static void mp_mul(int P, const double *x, const double *y, double *r) { mp_mul_v(P, 0, x, y, r); }

static int mp_is_zero(int P, const double *x)
{
    for (int c = 0; c < P; ++c)
        if (x[c] != 0.0)
            return 0;
    return 1;
}

static int mp_is_one(int P, const double *x)
{
    if (x[0] != 1.0)
        return 0;
    for (int c = 1; c < P; ++c)
        if (x[c] != 0.0)
            return 0;
    return 1;
}

static int is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }

/* op(A)(i, l) of a column-major component-plane matrix. */
static void load_op(int P, char t, const double *A, int64_t ld, int64_t ps,
                    int64_t i, int64_t l, double *out)
{
    int64_t off = is_trans(t) ? (l + i * ld) : (i + l * ld);
    for (int c = 0; c < P; ++c)
        out[c] = A[c * ps + off];
}

/* ------------------------------------------------------------------------ */
/* Exported element-wise operations and primitives (for pinning).           */
/* ------------------------------------------------------------------------ */

/* r[i] = x[i] op y[i] for i < n; planes at the given strides.  op: 0 add,
 * 1 mul, 2 the accurate TD addition (P == 3), 3 TDmulq (P == 3).  Returns -1
 * for an op that the precision does not have. */
EXPORT int ref_vec(int P, int op, int64_t n, const double *x, int64_t sx,
                   const double *y, int64_t sy, double *r, int64_t sr)
{
    if (op < 0 || op > 3 || (op >= 2 && P != 3))
        return -1;
    for (int64_t i = 0; i < n; ++i) {
        double a[4], b[4], o[4];
        for (int c = 0; c < P; ++c) {
            a[c] = x[c * sx + i];
            b[c] = y[c * sy + i];
        }
        if (op == 0)
            mp_add(P, a, b, o);
        else if (op == 1)
            mp_mul(P, a, b, o);
        else if (op == 2)
            td_add_acc(a, b, o);
        else
            td_mulq(a, b, o);
        for (int c = 0; c < P; ++c)
            r[c * sr + i] = o[c];
    }
    return 0;
}

/* Primitive under test, applied to n argument tuples stored argument-major
 * (in[a * n + i]); results stored result-major (out[q * n + i]).
 *   0 quick_two_sum(a,b)->(s,e)   1 two_sum(a,b)->(s,e)
 *   2 two_prod(a,b)->(p,e)        3 three_sum(a,b,c)->(a,b,c)
 *   4 three_sum2(a,b,c)->(a,b)    5 vec_sum(x0..x3)->(e0..e3)
 *   6 vseb2(e0,e1,e2)->(r0,r1)    7 renorm4(c0..c4)->(r0..r3)
 *   8 vseb3(e0..e5)->(r0,r1,r2)   9 vec_sum(x0..x2)->(e0..e2)
 *  10 merge(x0,x1,x2,y0,y1,y2)->(z0..z5) */
EXPORT int ref_prim(int which, int64_t n, const double *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double a[6], o[6];
        switch (which) {
        case 0:
            quick_two_sum(in[i], in[n + i], &o[0], &o[1]);
            out[i] = o[0]; out[n + i] = o[1];
            break;
        case 1:
            two_sum(in[i], in[n + i], &o[0], &o[1]);
            out[i] = o[0]; out[n + i] = o[1];
            break;
        case 2:
            two_prod(in[i], in[n + i], &o[0], &o[1]);
            out[i] = o[0]; out[n + i] = o[1];
            break;
        case 3:
            a[0] = in[i]; a[1] = in[n + i]; a[2] = in[2 * n + i];
            three_sum(&a[0], &a[1], &a[2]);
            for (int q = 0; q < 3; ++q) out[q * n + i] = a[q];
            break;
        case 4:
            a[0] = in[i]; a[1] = in[n + i]; a[2] = in[2 * n + i];
            three_sum2(&a[0], &a[1], a[2]);
            out[i] = a[0]; out[n + i] = a[1];
            break;
        case 5:
            for (int q = 0; q < 4; ++q) a[q] = in[q * n + i];
            vec_sum(a, 4, o);
            for (int q = 0; q < 4; ++q) out[q * n + i] = o[q];
            break;
        case 6:
            for (int q = 0; q < 3; ++q) a[q] = in[q * n + i];
            vseb(a, 3, o, 2);
            out[i] = o[0]; out[n + i] = o[1];
            break;
        case 7:
            renorm4(in[i], in[n + i], in[2 * n + i], in[3 * n + i], in[4 * n + i], o);
            for (int q = 0; q < 4; ++q) out[q * n + i] = o[q];
            break;
        case 8:
            for (int q = 0; q < 6; ++q) a[q] = in[q * n + i];
            vseb(a, 6, o, 3);
            for (int q = 0; q < 3; ++q) out[q * n + i] = o[q];
            break;
        case 9:
            for (int q = 0; q < 3; ++q) a[q] = in[q * n + i];
            vec_sum(a, 3, o);
            for (int q = 0; q < 3; ++q) out[q * n + i] = o[q];
            break;
        case 10:
            for (int q = 0; q < 6; ++q) a[q] = in[q * n + i];
            merge_mag(&a[0], 3, &a[3], 3, o);
            for (int q = 0; q < 6; ++q) out[q * n + i] = o[q];
            break;
        default:
            return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3, eqn (1): C = alpha op(A) op(B) + beta C, canonical order.        */
/* ------------------------------------------------------------------------ */

/* The paper computes c_ij as the sum over k of a_ik b_kj (eqn (1)) and leaves
 * the in-block order open.  Reading: for every entry, one running sum
 * acc = 0; for l = 0..k-1 ascending: acc = ADD(acc, MUL(a_il, b_lj)); then
 *   beta == 0:          c = MUL(alpha, acc)            (C is not read)
 *   otherwise:          c = ADD(MUL(alpha, acc), MUL(beta, c_old))
 *   alpha == 0 or k==0: c = beta == 0 ? 0 : MUL(beta, c_old)
 * and nothing is written when m == 0, n == 0, or (alpha == 0 or k == 0) and
 * beta == 1.  Only rows row0 <= i < row1 and columns col0 <= j < col1 are
 * computed (a negative end means "to the last"). */
static void epilogue(int P, int variant, const double *alpha, const double *acc,
                     const double *beta, double *c_io, int alpha_or_k_zero)
{
    double t1[4], t2[4];
    int beta_zero = mp_is_zero(P, beta);
    if (alpha_or_k_zero) {
        if (beta_zero) {
            for (int c = 0; c < P; ++c) c_io[c] = 0.0;
        } else {
            mp_mul_v(P, variant, beta, c_io, t2);
            for (int c = 0; c < P; ++c) c_io[c] = t2[c];
        }
        return;
    }
    mp_mul_v(P, variant, alpha, acc, t1);
    if (beta_zero) {
        for (int c = 0; c < P; ++c) c_io[c] = t1[c];
    } else {
        mp_mul_v(P, variant, beta, c_io, t2);
        mp_add_v(P, variant, t1, t2, c_io);
    }
}

/* The GEMM with the TD operations chosen by `variant` (0 for DD and QD). */
EXPORT int ref_gemm_v(int P, int variant, char ta, char tb, int64_t m, int64_t n, int64_t k,
                      const double *alpha, const double *A, int64_t lda, int64_t sa,
                      const double *B, int64_t ldb, int64_t sb, const double *beta,
                      double *C, int64_t ldc, int64_t sc, int64_t row0, int64_t row1,
                      int64_t col0, int64_t col1, int nthreads)
{
    if (P < 2 || P > 4)
        return -1;
    if (variant < 0 || variant > 3 || (variant != 0 && P != 3))
        return -2;
    if (row1 < 0 || row1 > m)
        row1 = m;
    if (row0 < 0)
        row0 = 0;
    if (col1 < 0 || col1 > n)
        col1 = n;
    if (col0 < 0)
        col0 = 0;
    int az = mp_is_zero(P, alpha) || k == 0;
    if (m == 0 || n == 0 || (az && mp_is_one(P, beta)))
        return 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    int64_t rows = row1 - row0, cols = col1 - col0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t idx = 0; idx < rows * cols; ++idx) {
        int64_t i = row0 + idx % rows;
        int64_t j = col0 + idx / rows;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (!az) {
            for (int64_t l = 0; l < k; ++l) {
                double a[4], b[4], p[4], t[4];
                load_op(P, ta, A, lda, sa, i, l, a);
                load_op(P, tb == 'N' || tb == 'n' ? 'T' : 'N', B, ldb, sb, j, l, b);
                mp_mul_v(P, variant, a, b, p);
                mp_add_v(P, variant, acc, p, t);
                for (int c = 0; c < P; ++c) acc[c] = t[c];
            }
        }
        double cv[4];
        for (int c = 0; c < P; ++c)
            cv[c] = C[c * sc + i + j * ldc];
        epilogue(P, variant, alpha, acc, beta, cv, az);
        for (int c = 0; c < P; ++c)
            C[c * sc + i + j * ldc] = cv[c];
    }
    return 0;
}

EXPORT int ref_gemm(int P, char ta, char tb, int64_t m, int64_t n, int64_t k,
                    const double *alpha, const double *A, int64_t lda, int64_t sa,
                    const double *B, int64_t ldb, int64_t sb, const double *beta,
                    double *C, int64_t ldc, int64_t sc, int64_t row0, int64_t row1,
                    int64_t col0, int64_t col1, int nthreads)
{
    return ref_gemm_v(P, 0, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc,
                      row0, row1, col0, col1, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Exact integers and their rounding into P components (used by both split  */
/* forms): a 512-bit two's complement integer X, and the components of      */
/* X 2^e by repeated round-to-nearest (ties to even) of the exact remainder. */
/* ------------------------------------------------------------------------ */

#define BIG_LIMBS 16          /* 512-bit two's complement, 32-bit limbs */

typedef struct {
    uint32_t w[BIG_LIMBS];    /* little-endian */
} big;

static void big_set_i64(big *a, int64_t v)
{
    uint64_t u = (uint64_t)v;
    a->w[0] = (uint32_t)u;
    a->w[1] = (uint32_t)(u >> 32);
    uint32_t ext = v < 0 ? 0xffffffffu : 0u;
    for (int i = 2; i < BIG_LIMBS; ++i) a->w[i] = ext;
}

static int big_neg_p(const big *a) { return (a->w[BIG_LIMBS - 1] >> 31) != 0; }

static void big_add(big *a, const big *b)
{
    uint64_t c = 0;
    for (int i = 0; i < BIG_LIMBS; ++i) {
        uint64_t t = (uint64_t)a->w[i] + b->w[i] + c;
        a->w[i] = (uint32_t)t;
        c = t >> 32;
    }
}

static void big_negate(big *a)
{
    uint64_t c = 1;
    for (int i = 0; i < BIG_LIMBS; ++i) {
        uint64_t t = (uint64_t)(~a->w[i]) + c;
        a->w[i] = (uint32_t)t;
        c = t >> 32;
    }
}

static void big_shl(big *a, int sh)     /* 0 <= sh < 32 */
{
    if (sh == 0)
        return;
    for (int i = BIG_LIMBS - 1; i > 0; --i)
        a->w[i] = (a->w[i] << sh) | (a->w[i - 1] >> (32 - sh));
    a->w[0] <<= sh;
}

static int big_top_bit(const big *a)    /* of a non-negative value; -1 if zero */
{
    for (int i = BIG_LIMBS - 1; i >= 0; --i)
        if (a->w[i])
            return 32 * i + 31 - __builtin_clz(a->w[i]);
    return -1;
}

static int big_bit(const big *a, int b) { return (a->w[b >> 5] >> (b & 31)) & 1; }

/* bits [lo, lo + 53) of a non-negative value as an integer */
static uint64_t big_bits53(const big *a, int lo)
{
    uint64_t r = 0;
    for (int b = lo + 52; b >= lo; --b)
        r = (r << 1) | (uint64_t)(b >= 0 ? big_bit(a, b) : 0);
    return r;
}

/* a -= q 2^sh for a non-negative a, q < 2^54 */
static void big_sub_shifted(big *a, uint64_t q, int sh)
{
    big t;
    memset(&t, 0, sizeof t);
    for (int b = 0; b < 54; ++b)
        if ((q >> b) & 1) {
            int pos = b + sh;
            t.w[pos >> 5] |= 1u << (pos & 31);
        }
    big_negate(&t);
    big_add(a, &t);
}

/* Components c_0..c_{P-1} of X 2^e: c_0 = RN(X 2^e), then RN of the exact
 * remainder, and so on (round to nearest, ties to even). */
static void big_to_components(int P, const big *X, int e, double *c)
{
    big m = *X;
    int neg = big_neg_p(&m);
    if (neg)
        big_negate(&m);
    for (int q = 0; q < P; ++q) {
        int h = big_top_bit(&m);
        if (h < 0) {
            c[q] = 0.0;
            continue;
        }
        if (h <= 52) {
            uint64_t v = big_bits53(&m, 0);
            c[q] = (neg ? -1.0 : 1.0) * ldexp((double)v, e);
            memset(&m, 0, sizeof m);
            continue;
        }
        int sh = h - 52;
        uint64_t v = big_bits53(&m, sh);
        /* rounding: guard bit sh-1, sticky below */
        int guard = big_bit(&m, sh - 1);
        int sticky = 0;
        for (int b = 0; b < sh - 1 && !sticky; ++b)
            sticky = big_bit(&m, b);
        if (guard && (sticky || (v & 1)))
            v += 1;
        c[q] = (neg ? -1.0 : 1.0) * ldexp((double)v, sh + e);
        /* remainder m - v 2^sh, which may be negative after rounding up */
        big_sub_shifted(&m, v, sh);
        if (big_neg_p(&m)) {
            big_negate(&m);
            neg = !neg;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Split (Ozaki-style) form: each operand entry is scaled by a power of two */
/* per row of op(A) / column of op(B) and cut into s signed 7-bit digits;   */
/* the digit products are exact integers, summed per anti-diagonal         */
/*   S_d = sum_{p+q=d} sum_l d_p(a_il) d_q(b_lj),  d = 2..s+1,             */
/* (the triangle p + q <= s + 1 of digit pairs), then recombined exactly:  */
/*   X_ij = sum_d S_d 128^(s+1-d)   (exact integer, Horner in base 128),   */
/*   value = X_ij 2^(E_i + F_j - 7 (s+1)),                                 */
/* rounded once into P components (repeated round-to-nearest of the exact  */
/* remainder), then the epilogue.  This form is not in the paper; it        */
/* reaches the paper's product by a different route and is held to the     */
/* same componentwise error bound.                                          */
/* ------------------------------------------------------------------------ */

/* Scale exponent of a row/column whose largest leading component has
 * magnitude M: E = e + 1 with M = f 2^e, f in [1/2, 1), so that every entry
 * divided by 2^E lies in (-1/2, 1/2).  An all-zero row/column gets E = 0. */
static int32_t scale_exponent(double M)
{
    if (M == 0.0)
        return 0;
    int e;
    frexp(M, &e);
    return (int32_t)(e + 1);
}

/* Digits of x = value / 2^E (|x| < 1/2), p = 1..s:
 *   re-sum the remainder with VecSum so its first component carries its
 *   leading bits; d_p = rint(r0 * 2^(7p)); r0 = (r0 * 2^(7p) - d_p) * 2^(-7p).
 * Every step is exact, |d_p| <= 64, and the remainder after s digits is at
 * most 2^(-7s-1) (1 + 2^-40) in magnitude. */
static void slice_one(int P, int s, const double *v, int32_t E, int8_t *digits, int64_t dstride)
{
    double r[4];
    for (int c = 0; c < P; ++c)
        r[c] = ldexp(v[c], -E);
    for (int p = 1; p <= s; ++p) {
        vec_sum(r, P, r);
        double y = ldexp(r[0], 7 * p);
        double d = nearbyint(y);
        r[0] = ldexp(y - d, -7 * p);
        digits[(int64_t)(p - 1) * dstride] = (int8_t)d;
    }
}

/* Exponents of the rows of op(A) (count = m) or, with is_b, the columns of
 * op(B) (count = n); k is the inner dimension. */
EXPORT void ref_split_exponents(int P, char t, int is_b, int64_t count, int64_t k,
                                const double *X, int64_t ld, int64_t ps, int32_t *E)
{
    (void)P;
    for (int64_t i = 0; i < count; ++i) {
        double M = 0.0;
        for (int64_t l = 0; l < k; ++l) {
            double v[4];
            if (!is_b)
                load_op(1, t, X, ld, ps, i, l, v);
            else
                load_op(1, (t == 'N' || t == 'n') ? 'T' : 'N', X, ld, ps, i, l, v);
            double a = fabs(v[0]);
            if (a > M)
                M = a;
        }
        E[i] = scale_exponent(M);
    }
}

/* Digits of op(A) rows / op(B) columns: D[(p-1) * count * k + i * k + l]. */
EXPORT void ref_split_slices(int P, int s, char t, int is_b, int64_t count, int64_t k,
                             const double *X, int64_t ld, int64_t ps, const int32_t *E,
                             int8_t *D)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        for (int64_t l = 0; l < k; ++l) {
            double v[4];
            if (!is_b)
                load_op(P, t, X, ld, ps, i, l, v);
            else
                load_op(P, (t == 'N' || t == 'n') ? 'T' : 'N', X, ld, ps, i, l, v);
            slice_one(P, s, v, E[i], D + i * k + l, count * k);
        }
}

/* Exact recombination of one entry's anti-diagonal sums S[d-2], d = 2..s+1:
 * X = sum_d S_d 128^(s+1-d) as an exact integer (Horner in base 128), then
 * the components of X 2^(ef - 7 (s+1)), rounded once. */
static void split_recombine(int P, int s, const int64_t *S, int32_t ef, double *acc)
{
    big X;
    big_set_i64(&X, 0);
    for (int d = 2; d <= s + 1; ++d) {
        big t;
        big_shl(&X, 7);
        big_set_i64(&t, S[d - 2]);
        big_add(&X, &t);
    }
    big_to_components(P, &X, ef - 7 * (s + 1), acc);
}

/* The recombination alone, for pinning: S holds `count` rows of s sums
 * (S[r * s + d - 2]), ef the row's E_i + F_j; out[r * P + c]. */
EXPORT int ref_split_recombine(int P, int s, int64_t count, const int64_t *S, const int32_t *ef,
                               double *out)
{
    if (P < 2 || P > 4 || s < 1 || s > 64)
        return -1;
    for (int64_t r = 0; r < count; ++r)
        split_recombine(P, s, S + r * s, ef[r], out + r * P);
    return 0;
}

/* Whole split-form GEMM for rows row0 <= i < row1 and columns col0 <= j <
 * col1 (negative end: to the last).  Optional debug outputs (NULL to skip):
 * E (m), F (n), S (s planes of m x n int64, column-major; only the computed
 * block written). */
EXPORT int ref_gemm_split(int P, int s, char ta, char tb, int64_t m, int64_t n, int64_t k,
                          const double *alpha, const double *A, int64_t lda, int64_t sa,
                          const double *B, int64_t ldb, int64_t sb, const double *beta,
                          double *C, int64_t ldc, int64_t sc, int64_t row0, int64_t row1,
                          int64_t col0, int64_t col1, int nthreads, int32_t *E_out,
                          int32_t *F_out, int64_t *S_out)
{
    if (P < 2 || P > 4 || s < 1 || s > 64)
        return -1;
    if (row1 < 0 || row1 > m)
        row1 = m;
    if (row0 < 0)
        row0 = 0;
    if (col1 < 0 || col1 > n)
        col1 = n;
    if (col0 < 0)
        col0 = 0;
    int az = mp_is_zero(P, alpha) || k == 0;
    if (m == 0 || n == 0 || (az && mp_is_one(P, beta)))
        return 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    int64_t rows = row1 - row0, cols = col1 - col0;
    int32_t *E = (int32_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int32_t));
    int32_t *F = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int8_t *DA = NULL, *DB = NULL;
    if (!az) {
        DA = (int8_t *)malloc((size_t)s * rows * k);
        DB = (int8_t *)malloc((size_t)s * cols * k);
        /* rows of op(A) in [row0, row1), columns of op(B) in [col0, col1) */
        const double *Ab = A + (is_trans(ta) ? row0 * lda : row0);
        const double *Bb = B + (is_trans(tb) ? col0 : col0 * ldb);
        ref_split_exponents(P, ta, 0, rows, k, Ab, lda, sa, E + row0);
        ref_split_exponents(P, tb, 1, cols, k, Bb, ldb, sb, F + col0);
        ref_split_slices(P, s, ta, 0, rows, k, Ab, lda, sa, E + row0, DA);
        ref_split_slices(P, s, tb, 1, cols, k, Bb, ldb, sb, F + col0, DB);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t idx = 0; idx < rows * cols; ++idx) {
        int64_t ii = idx % rows, i = row0 + ii;
        int64_t jj = idx / rows, j = col0 + jj;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (!az) {
            int64_t S[64];
            for (int d = 2; d <= s + 1; ++d) {
                int64_t sum = 0;
                for (int p = 1; p <= d - 1; ++p) {
                    int q = d - p;
                    const int8_t *da = DA + (int64_t)(p - 1) * rows * k + ii * k;
                    const int8_t *db = DB + (int64_t)(q - 1) * cols * k + jj * k;
                    for (int64_t l = 0; l < k; ++l)
                        sum += (int64_t)da[l] * (int64_t)db[l];
                }
                S[d - 2] = sum;
                if (S_out)
                    S_out[(int64_t)(d - 2) * m * n + i + j * m] = sum;
            }
            split_recombine(P, s, S, E[i] + F[j], acc);
        }
        double cv[4];
        for (int c = 0; c < P; ++c)
            cv[c] = C[c * sc + i + j * ldc];
        epilogue(P, 0, alpha, acc, beta, cv, az);
        for (int c = 0; c < P; ++c)
            C[c * sc + i + j * ldc] = cv[c];
    }
    if (E_out)
        memcpy(E_out + row0, E + row0, (size_t)rows * sizeof(int32_t));
    if (F_out)
        memcpy(F_out + col0, F + col0, (size_t)cols * sizeof(int32_t));
    free(E);
    free(F);
    free(DA);
    free(DB);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Strassen's method (Sec. 3, Fig. 5): for even dimensions, op(A), op(B) and */
/* C are cut into 2 x 2 blocks and the product is formed from seven block   */
/* products, recursively for `levels` levels; the blocks at the bottom are  */
/* multiplied in the canonical order above.  The paper's figure with the    */
/* formulas is not reproduced; the reading is Strassen's original scheme:   */
/*   M1 = (A11 + A22)(B11 + B22)   M2 = (A21 + A22) B11                     */
/*   M3 = A11 (B12 - B22)          M4 = A22 (B21 - B11)                     */
/*   M5 = (A11 + A12) B22          M6 = (A21 - A11)(B11 + B12)              */
/*   M7 = (A12 - A22)(B21 + B22)                                            */
/*   C11 = M1 + M4 - M5 + M7       C12 = M3 + M5                            */
/*   C21 = M2 + M4                 C22 = M1 - M2 + M3 + M6                  */
/* Sums are evaluated left to right; x - y is ADD(x, -y) with -y the exact  */
/* componentwise negation.  The product P = op(A) op(B) then goes through   */
/* the epilogue of the canonical GEMM (alpha, beta).                        */
/* ------------------------------------------------------------------------ */

/* A dense matrix view in op space: element (i, j) of component c is at
 * p[c * ps + (t ? j + i * ld : i + j * ld)]. */
typedef struct {
    double *p;
    int64_t ld, ps;
    int t;
} mview;

static mview mv_block(mview v, int64_t bi, int64_t bj, int64_t h, int64_t w)
{
    /* block (bi, bj) of height h and width w, in op space */
    mview r = v;
    r.p = v.t ? v.p + bj * w + bi * h * v.ld : v.p + bi * h + bj * w * v.ld;
    return r;
}

static void mv_get(int P, mview v, int64_t i, int64_t j, double *x)
{
    int64_t off = v.t ? j + i * v.ld : i + j * v.ld;
    for (int c = 0; c < P; ++c)
        x[c] = v.p[c * v.ps + off];
}

static void mv_set(int P, mview v, int64_t i, int64_t j, const double *x)
{
    int64_t off = v.t ? j + i * v.ld : i + j * v.ld;
    for (int c = 0; c < P; ++c)
        v.p[c * v.ps + off] = x[c];
}

/* R = X + sign * Y over h x w (sign = +1 or -1; -Y negated exactly). */
static void mv_addsub(int P, mview X, mview Y, int sign, mview R, int64_t h, int64_t w)
{
    for (int64_t j = 0; j < w; ++j)
        for (int64_t i = 0; i < h; ++i) {
            double x[4], y[4], r[4];
            mv_get(P, X, i, j, x);
            mv_get(P, Y, i, j, y);
            if (sign < 0)
                for (int c = 0; c < P; ++c) y[c] = -y[c];
            mp_add(P, x, y, r);
            mv_set(P, R, i, j, r);
        }
}

static mview mv_alloc(int P, int64_t h, int64_t w)
{
    mview v;
    v.p = (double *)calloc((size_t)P * (size_t)(h * w > 0 ? h * w : 1), sizeof(double));
    v.ld = h > 0 ? h : 1;
    v.ps = h * w;
    v.t = 0;
    return v;
}

/* Out (h x w, op space) = X (h x q) * Y (q x w). */
static int strassen_rec(int P, int levels, int64_t h, int64_t w, int64_t q, mview X, mview Y,
                        mview Out)
{
    if (levels == 0) {
        double one[4] = {1.0, 0.0, 0.0, 0.0}, zero[4] = {0.0, 0.0, 0.0, 0.0};
        return ref_gemm(P, X.t ? 'T' : 'N', Y.t ? 'T' : 'N', h, w, q, one, X.p, X.ld, X.ps,
                        Y.p, Y.ld, Y.ps, zero, Out.p, Out.ld, Out.ps, 0, -1, 0, -1, 0);
    }
    int64_t a = h / 2, b = w / 2, c = q / 2;
    mview A11 = mv_block(X, 0, 0, a, c), A12 = mv_block(X, 0, 1, a, c);
    mview A21 = mv_block(X, 1, 0, a, c), A22 = mv_block(X, 1, 1, a, c);
    mview B11 = mv_block(Y, 0, 0, c, b), B12 = mv_block(Y, 0, 1, c, b);
    mview B21 = mv_block(Y, 1, 0, c, b), B22 = mv_block(Y, 1, 1, c, b);
    mview C11 = mv_block(Out, 0, 0, a, b), C12 = mv_block(Out, 0, 1, a, b);
    mview C21 = mv_block(Out, 1, 0, a, b), C22 = mv_block(Out, 1, 1, a, b);
    mview SA = mv_alloc(P, a, c), SB = mv_alloc(P, c, b), M[7];
    for (int i = 0; i < 7; ++i)
        M[i] = mv_alloc(P, a, b);
    int rc = 0;
    mv_addsub(P, A11, A22, 1, SA, a, c);
    mv_addsub(P, B11, B22, 1, SB, c, b);
    rc |= strassen_rec(P, levels - 1, a, b, c, SA, SB, M[0]);
    mv_addsub(P, A21, A22, 1, SA, a, c);
    rc |= strassen_rec(P, levels - 1, a, b, c, SA, B11, M[1]);
    mv_addsub(P, B12, B22, -1, SB, c, b);
    rc |= strassen_rec(P, levels - 1, a, b, c, A11, SB, M[2]);
    mv_addsub(P, B21, B11, -1, SB, c, b);
    rc |= strassen_rec(P, levels - 1, a, b, c, A22, SB, M[3]);
    mv_addsub(P, A11, A12, 1, SA, a, c);
    rc |= strassen_rec(P, levels - 1, a, b, c, SA, B22, M[4]);
    mv_addsub(P, A21, A11, -1, SA, a, c);
    mv_addsub(P, B11, B12, 1, SB, c, b);
    rc |= strassen_rec(P, levels - 1, a, b, c, SA, SB, M[5]);
    mv_addsub(P, A12, A22, -1, SA, a, c);
    mv_addsub(P, B21, B22, 1, SB, c, b);
    rc |= strassen_rec(P, levels - 1, a, b, c, SA, SB, M[6]);
    /* C11 = M1 + M4 - M5 + M7, C12 = M3 + M5, C21 = M2 + M4, C22 = M1 - M2 + M3 + M6 */
    mv_addsub(P, M[0], M[3], 1, C11, a, b);
    mv_addsub(P, C11, M[4], -1, C11, a, b);
    mv_addsub(P, C11, M[6], 1, C11, a, b);
    mv_addsub(P, M[2], M[4], 1, C12, a, b);
    mv_addsub(P, M[1], M[3], 1, C21, a, b);
    mv_addsub(P, M[0], M[1], -1, C22, a, b);
    mv_addsub(P, C22, M[2], 1, C22, a, b);
    mv_addsub(P, C22, M[5], 1, C22, a, b);
    free(SA.p);
    free(SB.p);
    for (int i = 0; i < 7; ++i)
        free(M[i].p);
    return rc;
}

/* C = alpha op(A) op(B) + beta C with the product from `levels` levels of
 * Strassen's method; m, n, k must be multiples of 2^levels (else -2). */
EXPORT int ref_gemm_strassen(int P, int levels, char ta, char tb, int64_t m, int64_t n, int64_t k,
                             const double *alpha, const double *A, int64_t lda, int64_t sa,
                             const double *B, int64_t ldb, int64_t sb, const double *beta,
                             double *C, int64_t ldc, int64_t sc)
{
    if (P < 2 || P > 4 || levels < 0)
        return -1;
    int64_t unit = (int64_t)1 << levels;
    if (m % unit || n % unit || k % unit)
        return -2;
    int az = mp_is_zero(P, alpha) || k == 0;
    if (m == 0 || n == 0 || (az && mp_is_one(P, beta)))
        return 0;
    mview X = {(double *)A, lda, sa, is_trans(ta)}, Y = {(double *)B, ldb, sb, is_trans(tb)};
    mview PR = mv_alloc(P, m, n);
    int rc = az ? 0 : strassen_rec(P, levels, m, n, k, X, Y, PR);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double acc[4], cv[4];
            mv_get(P, PR, i, j, acc);
            for (int c = 0; c < P; ++c)
                cv[c] = C[c * sc + i + j * ldc];
            epilogue(P, 0, alpha, acc, beta, cv, az);
            for (int c = 0; c < P; ++c)
                C[c * sc + i + j * ldc] = cv[c];
        }
    free(PR.p);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* BLAS-1/2 in DD/TD/QD (the vector kernels the paper lists beside its      */
/* Strassen code, Sec. 4).  Readings:                                        */
/*   axpy: y_i = ADD(MUL(alpha, x_i), y_i);                                  */
/*   gemv: y = alpha op(A) x + beta y, each entry in the canonical GEMM      */
/*         order, i.e. exactly the GEMM with one column;                     */
/*   dot:  a 64-ary tree in a fixed order: the n products are taken in       */
/*         blocks of 64 consecutive terms, each block summed from zero in    */
/*         ascending order (acc = ADD(acc, MUL(x_i, y_i))); the block sums   */
/*         are again taken 64 at a time and summed the same way, until one   */
/*         value is left.  For n <= 64 this is the sequential chain.         */
/* ------------------------------------------------------------------------ */

#define DOT_FANIN 64

EXPORT int ref_axpy(int P, int64_t n, const double *alpha, const double *x, int64_t sx, double *y,
                    int64_t sy)
{
    if (P < 2 || P > 4)
        return -1;
    for (int64_t i = 0; i < n; ++i) {
        double a[4], b[4], t[4], r[4];
        for (int c = 0; c < P; ++c) {
            a[c] = x[c * sx + i];
            b[c] = y[c * sy + i];
        }
        mp_mul(P, alpha, a, t);
        mp_add(P, t, b, r);
        for (int c = 0; c < P; ++c)
            y[c * sy + i] = r[c];
    }
    return 0;
}

EXPORT int ref_dot(int P, int64_t n, const double *x, int64_t sx, const double *y, int64_t sy,
                   double *result)
{
    if (P < 2 || P > 4)
        return -1;
    if (n <= 0) {
        for (int c = 0; c < P; ++c) result[c] = 0.0;
        return 0;
    }
    /* level 0: block sums of products */
    int64_t cnt = (n + DOT_FANIN - 1) / DOT_FANIN;
    double *part = (double *)malloc((size_t)cnt * P * sizeof(double));
    for (int64_t b = 0; b < cnt; ++b) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t i = b * DOT_FANIN; i < n && i < (b + 1) * DOT_FANIN; ++i) {
            double a[4], e[4], p[4], t[4];
            for (int c = 0; c < P; ++c) {
                a[c] = x[c * sx + i];
                e[c] = y[c * sy + i];
            }
            mp_mul(P, a, e, p);
            mp_add(P, acc, p, t);
            for (int c = 0; c < P; ++c) acc[c] = t[c];
        }
        for (int c = 0; c < P; ++c) part[b * P + c] = acc[c];
    }
    /* higher levels: block sums of block sums */
    while (cnt > 1) {
        int64_t next = (cnt + DOT_FANIN - 1) / DOT_FANIN;
        for (int64_t b = 0; b < next; ++b) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int64_t i = b * DOT_FANIN; i < cnt && i < (b + 1) * DOT_FANIN; ++i) {
                double t[4];
                mp_add(P, acc, &part[i * P], t);
                for (int c = 0; c < P; ++c) acc[c] = t[c];
            }
            for (int c = 0; c < P; ++c) part[b * P + c] = acc[c];   /* b <= i: in place is safe */
        }
        cnt = next;
    }
    for (int c = 0; c < P; ++c) result[c] = part[c];
    free(part);
    return 0;
}

/* y (length rows of op(A)) = alpha op(A) x + beta y, A stored m x n (column-
 * major, planes at sa); x, y planes at sx, sy.  The GEMM with one column. */
EXPORT int ref_gemv(int P, char trans, int64_t m, int64_t n, const double *alpha, const double *A,
                    int64_t lda, int64_t sa, const double *x, int64_t sx, const double *beta,
                    double *y, int64_t sy)
{
    int t = is_trans(trans);
    int64_t rows = t ? n : m, inner = t ? m : n;
    return ref_gemm(P, trans, 'N', rows, 1, inner, alpha, A, lda, sa, x, inner > 0 ? inner : 1, sx,
                    beta, y, rows > 0 ? rows : 1, sy, 0, -1, 0, -1, 0);
}

/* ------------------------------------------------------------------------ */
/* Residue (CRT) form of the split product: the same digits as the split    */
/* form, but the product of the digit integers A'_il = sum_p d_p 128^(s-p)  */
/* and B'_lj is formed exactly over the full square of digit pairs:         */
/*   T_d = sum_{p+q=d} sum_l d_p(a_il) d_q(b_lj),  d = 2..2s,               */
/*   C'_ij = sum_d T_d 128^(2s-d)   (exact integer, Horner in base 128),   */
/*   value = C'_ij 2^(E_i + F_j - 14 s),                                   */
/* rounded to P components by repeated round-to-nearest (ties to even) of  */
/* the exact remainder, then the epilogue.  On the GPU the same integer is  */
/* obtained from its residues modulo pairwise coprime int8 moduli (one      */
/* INT8 matrix product per modulus) and the Chinese remainder theorem;      */
/* here it is the plain definition.                                         */
/* ------------------------------------------------------------------------ */

EXPORT int ref_gemm_crt(int P, int s, char ta, char tb, int64_t m, int64_t n, int64_t k,
                        const double *alpha, const double *A, int64_t lda, int64_t sa,
                        const double *B, int64_t ldb, int64_t sb, const double *beta,
                        double *C, int64_t ldc, int64_t sc, int64_t row0, int64_t row1,
                        int64_t col0, int64_t col1, int nthreads)
{
    if (P < 2 || P > 4 || s < 1 || s > 35)
        return -1;
    if (row1 < 0 || row1 > m)
        row1 = m;
    if (row0 < 0)
        row0 = 0;
    if (col1 < 0 || col1 > n)
        col1 = n;
    if (col0 < 0)
        col0 = 0;
    int az = mp_is_zero(P, alpha) || k == 0;
    if (m == 0 || n == 0 || (az && mp_is_one(P, beta)))
        return 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    int64_t rows = row1 - row0, cols = col1 - col0;
    int32_t *E = (int32_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int32_t));
    int32_t *F = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int8_t *DA = NULL, *DB = NULL;
    if (!az) {
        DA = (int8_t *)malloc((size_t)s * rows * k);
        DB = (int8_t *)malloc((size_t)s * cols * k);
        const double *Ab = A + (is_trans(ta) ? row0 * lda : row0);
        const double *Bb = B + (is_trans(tb) ? col0 : col0 * ldb);
        ref_split_exponents(P, ta, 0, rows, k, Ab, lda, sa, E + row0);
        ref_split_exponents(P, tb, 1, cols, k, Bb, ldb, sb, F + col0);
        ref_split_slices(P, s, ta, 0, rows, k, Ab, lda, sa, E + row0, DA);
        ref_split_slices(P, s, tb, 1, cols, k, Bb, ldb, sb, F + col0, DB);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t idx = 0; idx < rows * cols; ++idx) {
        int64_t ii = idx % rows, i = row0 + ii;
        int64_t jj = idx / rows, j = col0 + jj;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (!az) {
            big X;
            big_set_i64(&X, 0);
            for (int d = 2; d <= 2 * s; ++d) {
                int64_t T = 0;
                for (int p = 1; p <= s; ++p) {
                    int q = d - p;
                    if (q < 1 || q > s)
                        continue;
                    const int8_t *da = DA + (int64_t)(p - 1) * rows * k + ii * k;
                    const int8_t *db = DB + (int64_t)(q - 1) * cols * k + jj * k;
                    for (int64_t l = 0; l < k; ++l)
                        T += (int64_t)da[l] * (int64_t)db[l];
                }
                /* X = X 128 + T */
                big_shl(&X, 7);
                big t;
                big_set_i64(&t, T);
                big_add(&X, &t);
            }
            big_to_components(P, &X, E[i] + F[j] - 14 * s, acc);
        }
        double cv[4];
        for (int c = 0; c < P; ++c)
            cv[c] = C[c * sc + i + j * ldc];
        epilogue(P, 0, alpha, acc, beta, cv, az);
        for (int c = 0; c < P; ++c)
            C[c * sc + i + j * ldc] = cv[c];
    }
    free(E);
    free(F);
    free(DA);
    free(DB);
    return 0;
}

EXPORT int ref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
