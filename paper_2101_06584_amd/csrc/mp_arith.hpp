// mp_arith.hpp -- device-side double-double (P=2), triple-double (P=3) and
// quad-double (P=4) arithmetic for gfx950, built from error-free
// transformations on the FP64 vector ALUs.
//
// Every function reproduces, operation for operation, the sequences of the
// paper (Kouya, arXiv 2101.06584): Sec. 2.1 (QuickTwoSum, TwoSum, TwoProd),
// Algorithm 1 (DD add), Algorithm 2 (DD mul), Algorithm 4 (TD mul), Algorithm
// 5 (QD add, also the default TD add "TDaddq" with zero fourth components)
// and Algorithm 6 (QD mul), so a GEMM that keeps one sequential k-chain per
// entry is bitwise reproducible.  The data-dependent branches of VSEB(k) and
// Renorm are written as selects so a wavefront never diverges; the selected
// values are exactly those the branching form produces.  The GEMM inner step
// (tile_mac) adds a wave-uniform fast path for the common branch outcome.
//
// Compile with -ffp-contract=off: a contracted a*b+c would change results.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

namespace mpg {

template <int P>
struct mp {
    double c[P];
};

#define MPG_DEV __device__ __forceinline__

// ---- Sec. 2.1 ------------------------------------------------------------

// s = fl(a+b), e = b - (s - a); exact when exponent(a) >= exponent(b).
MPG_DEV void quick_two_sum(double a, double b, double& s, double& e) {
    double sum = a + b;
    e = b - (sum - a);
    s = sum;
}

// Knuth's TwoSum, its six operations in the order Algorithm 5 spells them
// out: s = a + b, v = s - a, u = s - v, w = a - u, u' = b - v, e = w + u'.
MPG_DEV void two_sum(double a, double b, double& s, double& e) {
    double sum = a + b;
    double v = sum - a;
    double u = sum - v;
    double w = a - u;
    double u2 = b - v;
    e = w + u2;
    s = sum;
}

// p = fl(ab), e = ab - p exactly via the fused multiply-add.
MPG_DEV void two_prod(double a, double b, double& p, double& e) {
    double prod = a * b;
    e = __builtin_fma(a, b, -prod);
    p = prod;
}

// (a, b, c) <- exact three-term re-sum (three TwoSums).
MPG_DEV void three_sum(double& a, double& b, double& c) {
    double t1, t2, t3;
    two_sum(a, b, t1, t2);
    two_sum(c, t1, a, t3);
    two_sum(t2, t3, b, c);
}

// (a, b) <- two leading terms; the two error terms rounded into b.
MPG_DEV void three_sum2(double& a, double& b, double c) {
    double t1, t2, t3;
    two_sum(a, b, t1, t2);
    two_sum(c, t1, a, t3);
    b = t2 + t3;
}

// Five terms to four (the renormalisation that Sec. 2 asks to be written as
// plain loops, so that it vectorises): a
// bottom-up QuickTwoSum pass, then a top-down pass in which a non-zero
// rounding error closes an output slot; when the third slot closes the last
// one takes the carry plus what remains.  Unrolled, slot writes by select.
MPG_DEV void renorm4(double c0, double c1, double c2, double c3, double c4,
                     double& r0, double& r1, double& r2, double& r3) {
    double s, e0, e1, e2, e3, e4;
    quick_two_sum(c3, c4, s, e4);
    quick_two_sum(c2, s, s, e3);
    quick_two_sum(c1, s, s, e2);
    quick_two_sum(c0, s, e0, e1);

    // pair (e0, e1) as pass 1 produced it
    bool k1 = (e1 != 0.0);
    r0 = k1 ? e0 : 0.0;
    r1 = 0.0;
    r2 = 0.0;
    r3 = 0.0;
    double carry = k1 ? e1 : e0;
    int j = k1 ? 1 : 0;

    double sv, t;
    quick_two_sum(carry, e2, sv, t);
    bool k2 = (t != 0.0);
    r0 = (k2 && j == 0) ? sv : r0;
    r1 = (k2 && j == 1) ? sv : r1;
    j += k2 ? 1 : 0;
    carry = k2 ? t : sv;

    quick_two_sum(carry, e3, sv, t);
    bool k3 = (t != 0.0);
    r0 = (k3 && j == 0) ? sv : r0;
    r1 = (k3 && j == 1) ? sv : r1;
    r2 = (k3 && j == 2) ? sv : r2;
    j += k3 ? 1 : 0;
    carry = k3 ? t : sv;
    bool done = (j == 3);

    // When the third slot closed at e3, the last slot is carry + e4, which is
    // exactly the sum half of this QuickTwoSum.
    quick_two_sum(carry, e4, sv, t);
    bool k4 = !done && (t != 0.0);
    r0 = (k4 && j == 0) ? sv : r0;
    r1 = (k4 && j == 1) ? sv : r1;
    r2 = (k4 && j == 2) ? sv : r2;
    j += k4 ? 1 : 0;
    carry = k4 ? t : sv;

    r0 = (j == 0) ? carry : r0;
    r1 = (j == 1) ? carry : r1;
    r2 = (j == 2) ? carry : r2;
    r3 = (j == 3) ? carry : r3;
}

// VSEB(2) on three terms (Sec. 2.3), as used by the TD product.  Cases of the
// two QuickTwoSums' error terms (t1, t2):
//   t1 != 0:           (s1, s2) with s2 from QuickTwoSum(t1, e3)
//   t1 == 0, t2 != 0:  (s2, t2) with s2 from QuickTwoSum(s1, e3)
//   t1 == 0, t2 == 0:  (s2, 0)
MPG_DEV void vseb2(double e1, double e2, double e3, double& r1, double& r2) {
    double s1, t1, s2, t2;
    quick_two_sum(e1, e2, s1, t1);
    bool k1 = (t1 != 0.0);
    double carry = k1 ? t1 : s1;
    quick_two_sum(carry, e3, s2, t2);
    bool k2 = (t2 != 0.0);
    r1 = k1 ? s1 : s2;
    r2 = k1 ? s2 : (k2 ? t2 : 0.0);
}

// ---- Algorithm 1 / Algorithm 2 -------------------------------------------

MPG_DEV mp<2> add(const mp<2>& x, const mp<2>& y) {
    double s, e;
    two_sum(x.c[0], y.c[0], s, e);
    double w = x.c[1] + y.c[1];
    e = e + w;
    mp<2> r;
    quick_two_sum(s, e, r.c[0], r.c[1]);
    return r;
}

MPG_DEV mp<2> mul(const mp<2>& x, const mp<2>& y) {
    double p1, p2;
    two_prod(x.c[0], y.c[0], p1, p2);
    double w1 = x.c[0] * y.c[1];
    double w2 = x.c[1] * y.c[0];
    double w3 = w1 + w2;
    p2 = p2 + w3;
    mp<2> r;
    quick_two_sum(p1, p2, r.c[0], r.c[1]);
    return r;
}

// ---- Algorithms 4, 5, 6: the terms before the final Renorm / VSEB(2) ------
//
// Algorithm 5 (QD add): its tail takes a fourth error term that the text never
// defines; read as the error of the fourth component pair's TwoSum, like the
// other three.
// Algorithm 6 (QD mul): a sum of the leading components that the algorithm
// computes first is overwritten before any use and is left out; the
// order-eps^3 terms are added one at a time in the paper's order, each a
// rounded multiply and a rounded add.
// Algorithm 4 (TD mul): b0..b2 are VecSum outputs, not operand components.

// TwoSum applied to N component pairs at once, each of its six operations
// over all pairs before the next (the form a vector unit runs it in).
template <int N>
MPG_DEV void two_sum_lanes(const double (&a)[N], const double (&b)[N], double (&s)[N], double (&e)[N]) {
    double v[N], u[N], w[N];
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] = a[i] + b[i];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = s[i] - a[i];
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = s[i] - v[i];
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = a[i] - u[i];
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = b[i] - v[i];
#pragma unroll
    for (int i = 0; i < N; ++i) e[i] = w[i] + u[i];
}

// Terms of the QD addition (Algorithm 5) before its Renorm (c0..c4).  Each
// pair of components x_i + y_i is added exactly (TwoSum: sum s_i, error t_i);
// the errors are then carried one level down: level 1 takes t_0 (one carry
// out), level 2 takes that carry and t_1 (ThreeSum, two carries out), level
// 3 takes one of them and t_2 (ThreeSum2, one carry out), and the fifth term
// collects the carries left over and t_3.
MPG_DEV void qd_add_terms(double x0, double x1, double x2, double x3, double y0, double y1,
                          double y2, double y3, double (&c)[5]) {
    const double x[4] = {x0, x1, x2, x3}, y[4] = {y0, y1, y2, y3};
    double sm[4], er[4];
    two_sum_lanes<4>(x, y, sm, er);
    double carry = er[0], carry2 = er[1];
    two_sum(sm[1], carry, sm[1], carry);
    three_sum(sm[2], carry, carry2);
    three_sum2(sm[3], carry, er[2]);
    c[0] = sm[0];
    c[1] = sm[1];
    c[2] = sm[2];
    c[3] = sm[3];
    c[4] = (carry + carry2) + er[3];
}

// qd_add_terms with zero fourth components (TDaddq), the same bits with four
// operations fewer.  The fourth pair's TwoSum is +0 + +0: sum and error +0.
// ThreeSum2 then starts with TwoSum(+0, carry): for finite carry its sum is
// carry + 0 (carry, or +0 for carry = -0), and its error is +0 whatever carry
// is: v = sum - 0 = sum, u = sum - v = +0, w = 0 - u = +0, u' = carry - v is
// +0, or -0 when carry = -0, and w + u' = +0.  So the error's four operations
// are dropped and ThreeSum2's last sum is +0 + t3, kept as such (it turns a
// -0 into +0, as the general form does).
MPG_DEV void td_add_terms(double x0, double x1, double x2, double y0, double y1, double y2,
                          double (&c)[5]) {
    const double x[3] = {x0, x1, x2}, y[3] = {y0, y1, y2};
    double sm[3], er[3];
    two_sum_lanes<3>(x, y, sm, er);
    double carry = er[0], carry2 = er[1];
    two_sum(sm[1], carry, sm[1], carry);
    three_sum(sm[2], carry, carry2);
    const double t1 = carry + 0.0;      // TwoSum(+0, carry)'s sum
    double s3, t3;
    two_sum(er[2], t1, s3, t3);
    c[0] = sm[0];
    c[1] = sm[1];
    c[2] = sm[2];
    c[3] = s3;
    c[4] = (0.0 + t3 + carry2) + 0.0;
}

// Terms of the QD product (Algorithm 6) before its Renorm (c0..c4).  The
// component products of order eps^0 to eps^2 (x_i y_j, i + j <= 2, taken
// as (0,0), (0,1), (1,0), (0,2), (1,1), (2,0)) are split exactly by TwoProd
// into p and q.  Order eps: ThreeSum of p01, p10 and q00.  Order eps^2: the
// carry of that sum with q01 and q10 (ThreeSum), and p02, p11, p20
// (ThreeSum); the two sums and their carries are combined by TwoSums into the
// order-eps^2 term and a lower one.  The order-eps^3 rest is added in rounded
// arithmetic: the products x_i y_(3-i) for i = 0..3 one at a time, then the
// errors q00, q02, q11, q20.
MPG_DEV void qd_mul_terms(const mp<4>& x, const mp<4>& y, double (&c)[5]) {
    // p_ij + q_ij = x_i y_j exactly
    double p00, q00, p01, q01, p10, q10, p02, q02, p11, q11, p20, q20;
    two_prod(x.c[0], y.c[0], p00, q00);
    two_prod(x.c[0], y.c[1], p01, q01);
    two_prod(x.c[1], y.c[0], p10, q10);
    two_prod(x.c[0], y.c[2], p02, q02);
    two_prod(x.c[1], y.c[1], p11, q11);
    two_prod(x.c[2], y.c[0], p20, q20);
    three_sum(p01, p10, q00);          // order eps: sum in p01, carries p10, q00
    three_sum(p10, q01, q10);          // the first carry with q01 and q10
    three_sum(p02, p11, p20);          // order-eps^2 products
    double hi, hi_err, mid, mid_err;
    two_sum(p10, p02, hi, hi_err);
    two_sum(q01, p11, mid, mid_err);
    double lo = q10 + p20;
    two_sum(mid, hi_err, mid, hi_err);
    lo = lo + (hi_err + mid_err);
    mid = mid + x.c[0] * y.c[3];       // order eps^3, rounded
    mid = mid + x.c[1] * y.c[2];
    mid = mid + x.c[2] * y.c[1];
    mid = mid + x.c[3] * y.c[0];
    mid = mid + q00;
    mid = mid + q02;
    mid = mid + q11;
    mid = mid + q20;
    c[0] = p00;
    c[1] = p01;
    c[2] = hi;
    c[3] = mid;
    c[4] = lo;
}

// Terms of Algorithm 4 before its VSEB(2): (e0, e1, e2, e3).
MPG_DEV void td_mul_terms(const mp<3>& x, const mp<3>& y, double (&e)[4]) {
    double z00u, z00l, z01u, z01l, z10u, z10l;
    two_prod(x.c[0], y.c[0], z00u, z00l);
    two_prod(x.c[0], y.c[1], z01u, z01l);
    two_prod(x.c[1], y.c[0], z10u, z10l);
    double b0, b1, b2, sv;
    two_sum(z01u, z10u, sv, b2);
    two_sum(z00l, sv, b0, b1);
    double c = __builtin_fma(x.c[1], y.c[1], b2);
    double z31 = __builtin_fma(x.c[0], y.c[2], z10l);
    double z32 = __builtin_fma(x.c[2], y.c[0], z01l);
    double z3 = z31 + z32;
    double s3 = c + z3;
    two_sum(b1, s3, sv, e[3]);
    two_sum(b0, sv, sv, e[2]);
    two_sum(z00u, sv, e[0], e[1]);
}

// ---- the finished operations ------------------------------------------------

MPG_DEV mp<4> add(const mp<4>& x, const mp<4>& y) {
    double t[5];
    qd_add_terms(x.c[0], x.c[1], x.c[2], x.c[3], y.c[0], y.c[1], y.c[2], y.c[3], t);
    mp<4> r;
    renorm4(t[0], t[1], t[2], t[3], t[4], r.c[0], r.c[1], r.c[2], r.c[3]);
    return r;
}

// TDaddq: the QD addition with zero fourth components, fourth output dropped.
MPG_DEV mp<3> add(const mp<3>& x, const mp<3>& y) {
    double t[5];
    td_add_terms(x.c[0], x.c[1], x.c[2], y.c[0], y.c[1], y.c[2], t);
    mp<3> r;
    double r3;
    renorm4(t[0], t[1], t[2], t[3], t[4], r.c[0], r.c[1], r.c[2], r3);
    (void)r3;
    return r;
}

MPG_DEV mp<4> mul(const mp<4>& x, const mp<4>& y) {
    double t[5];
    qd_mul_terms(x, y, t);
    mp<4> r;
    renorm4(t[0], t[1], t[2], t[3], t[4], r.c[0], r.c[1], r.c[2], r.c[3]);
    return r;
}

MPG_DEV mp<3> mul(const mp<3>& x, const mp<3>& y) {
    double e[4];
    td_mul_terms(x, y, e);
    mp<3> r;
    r.c[0] = e[0];
    vseb2(e[1], e[2], e[3], r.c[1], r.c[2]);
    return r;
}

// ---- Tile multiply-accumulate with a wave-uniform fast path ---------------
//
// The data-dependent branches of Renorm and VSEB(2) almost always take one
// path on non-degenerate data: every QuickTwoSum error of the second pass is
// non-zero, so each output slot closes in turn.  That path needs no selects:
//   Renorm:  r = (e0, s(e1+e2), s(t+e3), t' + e4)
//   VSEB(2): r = (s(e1+e2), s(t+e3))
// For a whole TM x TN register tile the terms before the final Renorm/VSEB are
// computed first; if every lane of the wave took the common path for every
// entry, its results are used, otherwise the select form recomputes the
// finish from the same terms.  Either way the values are exactly those of the
// general algorithm.

MPG_DEV bool renorm4_fast(double c0, double c1, double c2, double c3, double c4, double& r0,
                          double& r1, double& r2, double& r3) {
    double s, e0, e1, e2, e3, e4;
    quick_two_sum(c3, c4, s, e4);
    quick_two_sum(c2, s, s, e3);
    quick_two_sum(c1, s, s, e2);
    quick_two_sum(c0, s, e0, e1);
    double sv2, t2, sv3, t3;
    quick_two_sum(e1, e2, sv2, t2);
    quick_two_sum(t2, e3, sv3, t3);
    r0 = e0;
    r1 = sv2;
    r2 = sv3;
    r3 = t3 + e4;
    return (e1 != 0.0) && (t2 != 0.0) && (t3 != 0.0);
}

// The first three outputs of Renorm (all a TD result keeps): when the first
// two slots close, the third is sv3 if its error is non-zero and otherwise
// the sum of the carry sv3 with e4 (whether or not that sum then closes the
// slot, which only decides the dropped fourth output).  That sum is sv3
// itself when e4 = 0: with t2 != 0, sv3 = t2 + e3 is never -0, so adding
// +0 changes no bit.  In the TD product's accumulation e4 is zero in
// practice (the fourth components are zero) while t3 is zero about half of
// the time, so the fast path takes r2 = sv3 when t3 != 0 or e4 = 0 and
// leaves the rest (t3 = 0 with e4 != 0) to the general path.
MPG_DEV bool renorm3_fast(double c0, double c1, double c2, double c3, double c4, double& r0,
                          double& r1, double& r2) {
    double s, e0, e1, e2, e3, e4;
    quick_two_sum(c3, c4, s, e4);
    quick_two_sum(c2, s, s, e3);
    quick_two_sum(c1, s, s, e2);
    quick_two_sum(c0, s, e0, e1);
    double sv2, t2, sv3, t3;
    quick_two_sum(e1, e2, sv2, t2);
    quick_two_sum(t2, e3, sv3, t3);
    r0 = e0;
    r1 = sv2;
    r2 = sv3;
    return (e1 != 0.0) && (t2 != 0.0) && (t3 != 0.0 || e4 == 0.0);
}

MPG_DEV bool vseb2_fast(double e1, double e2, double e3, double& r1, double& r2) {
    double s1, t1, s2, t2;
    quick_two_sum(e1, e2, s1, t1);
    quick_two_sum(t1, e3, s2, t2);
    r1 = s1;
    r2 = s2;
    return t1 != 0.0;
}

// acc[r][c] = ADD(acc[r][c], MUL(a[r], b[c])) for a TM x TN tile.
template <int TM, int TN>
MPG_DEV void tile_mac(mp<2> (&acc)[TM][TN], const mp<2> (&a)[TM], const mp<2> (&b)[TN]) {
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[r][c] = add(acc[r][c], mul(a[r], b[c]));
}

template <int TM, int TN>
MPG_DEV void tile_mac(mp<4> (&acc)[TM][TN], const mp<4> (&a)[TM], const mp<4> (&b)[TN]) {
    double t[TM][TN][5];
    mp<4> prod[TM][TN];
    bool ok = true;
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) {
            qd_mul_terms(a[r], b[c], t[r][c]);
            ok = renorm4_fast(t[r][c][0], t[r][c][1], t[r][c][2], t[r][c][3], t[r][c][4],
                              prod[r][c].c[0], prod[r][c].c[1], prod[r][c].c[2], prod[r][c].c[3]) && ok;
        }
    if (!__all(ok)) {
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int c = 0; c < TN; ++c)
                renorm4(t[r][c][0], t[r][c][1], t[r][c][2], t[r][c][3], t[r][c][4], prod[r][c].c[0],
                        prod[r][c].c[1], prod[r][c].c[2], prod[r][c].c[3]);
    }
    ok = true;
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) {
            qd_add_terms(acc[r][c].c[0], acc[r][c].c[1], acc[r][c].c[2], acc[r][c].c[3],
                         prod[r][c].c[0], prod[r][c].c[1], prod[r][c].c[2], prod[r][c].c[3], t[r][c]);
            ok = renorm4_fast(t[r][c][0], t[r][c][1], t[r][c][2], t[r][c][3], t[r][c][4],
                              acc[r][c].c[0], acc[r][c].c[1], acc[r][c].c[2], acc[r][c].c[3]) && ok;
        }
    if (!__all(ok)) {
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int c = 0; c < TN; ++c)
                renorm4(t[r][c][0], t[r][c][1], t[r][c][2], t[r][c][3], t[r][c][4], acc[r][c].c[0],
                        acc[r][c].c[1], acc[r][c].c[2], acc[r][c].c[3]);
    }
}

template <int TM, int TN>
MPG_DEV void tile_mac(mp<3> (&acc)[TM][TN], const mp<3> (&a)[TM], const mp<3> (&b)[TN]) {
    double e[TM][TN][4];
    mp<3> prod[TM][TN];
    bool ok = true;
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) {
            td_mul_terms(a[r], b[c], e[r][c]);
            prod[r][c].c[0] = e[r][c][0];
            ok = vseb2_fast(e[r][c][1], e[r][c][2], e[r][c][3], prod[r][c].c[1], prod[r][c].c[2]) && ok;
        }
    if (!__all(ok)) {
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int c = 0; c < TN; ++c)
                vseb2(e[r][c][1], e[r][c][2], e[r][c][3], prod[r][c].c[1], prod[r][c].c[2]);
    }
    double t[TM][TN][5];
    ok = true;
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) {
            // TDaddq: Algorithm 5 with zero fourth components, fourth output dropped
            td_add_terms(acc[r][c].c[0], acc[r][c].c[1], acc[r][c].c[2], prod[r][c].c[0],
                         prod[r][c].c[1], prod[r][c].c[2], t[r][c]);
            ok = renorm3_fast(t[r][c][0], t[r][c][1], t[r][c][2], t[r][c][3], t[r][c][4],
                              acc[r][c].c[0], acc[r][c].c[1], acc[r][c].c[2]) && ok;
        }
    if (!__all(ok)) {
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int c = 0; c < TN; ++c) {
                double r3;
                renorm4(t[r][c][0], t[r][c][1], t[r][c][2], t[r][c][3], t[r][c][4], acc[r][c].c[0],
                        acc[r][c].c[1], acc[r][c].c[2], r3);
                (void)r3;
            }
    }
}

// ---- The other TD operations of Sec. 2.3 ---------------------------------
//
// The accurate TD addition (Algorithm 3) and TDmulq, which the paper measures
// against its defaults (TDaddq, Algorithm 4).  Selected per call through a
// variant: bit 0 the accurate addition, bit 1 TDmulq.

// Merge of two three-term expansions by decreasing magnitude: the two-pointer
// merge, x's head first when |x_i| >= |y_j|.  Written with selects (no
// run-time register indexing).
MPG_DEV void merge3(const mp<3>& x, const mp<3>& y, double (&z)[6]) {
    // the heads are shifted queues (hx0 = current head of x), so no value is
    // ever picked by a run-time index
    double hx0 = x.c[0], hx1 = x.c[1], hx2 = x.c[2];
    double hy0 = y.c[0], hy1 = y.c[1], hy2 = y.c[2];
    int nx = 3, ny = 3;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const bool take_x = (ny == 0) || (nx > 0 && fabs(hx0) >= fabs(hy0));
        z[k] = take_x ? hx0 : hy0;
        hx0 = take_x ? hx1 : hx0;
        hx1 = take_x ? hx2 : hx1;
        hy0 = take_x ? hy0 : hy1;
        hy1 = take_x ? hy1 : hy2;
        nx -= take_x ? 1 : 0;
        ny -= take_x ? 0 : 1;
    }
}

// VecSum over N terms: s = x[N-1]; (s, e[i+1]) = TwoSum(x[i], s) for
// i = N-2..0; e[0] = s.
template <int N>
MPG_DEV void vec_sum_n(const double (&x)[N], double (&e)[N]) {
    double s = x[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) two_sum(x[i], s, s, e[i + 1]);
    e[0] = s;
}

// VSEB(K) over N terms in select form: a top-down QuickTwoSum pass; a
// non-zero error closes the next output (the sum is the output, the error
// the new carry), a zero error keeps the sum as carry; after K outputs the
// rest is dropped; the carry fills the next open output at the end, later
// outputs are zero.
template <int N, int K>
MPG_DEV void vseb_n(const double (&e)[N], double (&r)[K]) {
#pragma unroll
    for (int q = 0; q < K; ++q) r[q] = 0.0;
    int j = 0;
    bool done = false;
    double carry = e[0];
#pragma unroll
    for (int i = 1; i < N; ++i) {
        double s, t;
        quick_two_sum(carry, e[i], s, t);
        const bool close = !done && (t != 0.0);
#pragma unroll
        for (int q = 0; q < K; ++q) r[q] = (close && j == q) ? s : r[q];
        carry = done ? carry : (close ? t : s);
        j += close ? 1 : 0;
        done = done || (j == K);
    }
#pragma unroll
    for (int q = 0; q < K; ++q) r[q] = (!done && j == q) ? carry : r[q];
}

// Algorithm 3: Merge, VecSum over the six terms, VSEB(3).
MPG_DEV mp<3> td_add_acc(const mp<3>& x, const mp<3>& y) {
    double z[6], e[6], r[3];
    merge3(x, y, z);
    vec_sum_n<6>(z, e);
    vseb_n<6, 3>(e, r);
    return mp<3>{{r[0], r[1], r[2]}};
}

// TDmulq: Algorithm 6 on (x0, x1, x2, 0) and (y0, y1, y2, 0), fourth output
// dropped.
MPG_DEV mp<3> td_mulq(const mp<3>& x, const mp<3>& y) {
    const mp<4> r = mul(mp<4>{{x.c[0], x.c[1], x.c[2], 0.0}}, mp<4>{{y.c[0], y.c[1], y.c[2], 0.0}});
    return mp<3>{{r.c[0], r.c[1], r.c[2]}};
}

// The precision's addition / multiplication under variant V (only TD has
// variants).
template <int V, int P>
MPG_DEV mp<P> add_v(const mp<P>& x, const mp<P>& y) {
    if constexpr (P == 3 && (V & 1) != 0) return td_add_acc(x, y);
    else return add(x, y);
}
template <int V, int P>
MPG_DEV mp<P> mul_v(const mp<P>& x, const mp<P>& y) {
    if constexpr (P == 3 && (V & 2) != 0) return td_mulq(x, y);
    else return mul(x, y);
}

// tile_mac under variant V: the fast-path tile routine for V == 0, the plain
// loop over add_v / mul_v otherwise.
template <int V, int TM, int TN, int P>
MPG_DEV void tile_mac_v(mp<P> (&acc)[TM][TN], const mp<P> (&a)[TM], const mp<P> (&b)[TN]) {
    if constexpr (V == 0) {
        tile_mac<TM, TN>(acc, a, b);
    } else {
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int c = 0; c < TN; ++c) acc[r][c] = add_v<V>(acc[r][c], mul_v<V>(a[r], b[c]));
    }
}

template <int P>
MPG_DEV mp<P> mp_zero() {
    mp<P> r;
#pragma unroll
    for (int q = 0; q < P; ++q) r.c[q] = 0.0;
    return r;
}

template <int P>
MPG_DEV bool mp_is_zero(const mp<P>& x) {
    bool z = true;
#pragma unroll
    for (int q = 0; q < P; ++q) z = z && (x.c[q] == 0.0);
    return z;
}

}  // namespace mpg
