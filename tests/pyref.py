"""A second, independent transcription of the paper's DD/TD/QD operations in
pure-Python binary64 (Python floats are IEEE binary64, round-to-nearest-even).
Python 3.10 has no math.fma, so fma is evaluated exactly with Fractions and
rounded once (int / int true division is correctly rounded).

Used only as a cross-check of the C oracle's transcription on small inputs;
the oracle's real pins are the exact-arithmetic tests.
"""
from __future__ import annotations

import math
from fractions import Fraction


def fma(a: float, b: float, c: float) -> float:
    r = Fraction(a) * Fraction(b) + Fraction(c)
    if r == 0:
        # IEEE exact-zero sign rule in round-to-nearest: -0 only when the
        # (zero) product and c are both -0; any other exact cancellation is +0
        prod_neg = (math.copysign(1.0, a) * math.copysign(1.0, b)) < 0
        prod_zero = a == 0.0 or b == 0.0
        c_neg = math.copysign(1.0, c) < 0
        if prod_zero and c == 0.0 and prod_neg and c_neg:
            return -0.0
        return 0.0
    return float(r)


def qts(a, b):
    s = a + b
    return s, b - (s - a)


def ts(a, b):
    s = a + b
    v = s - a
    u = s - v
    return s, (a - u) + (b - v)


def tp(a, b):
    p = a * b
    return p, fma(a, b, -p)


def three_sum(a, b, c):
    t1, t2 = ts(a, b)
    a2, t3 = ts(c, t1)
    b2, c2 = ts(t2, t3)
    return a2, b2, c2


def three_sum2(a, b, c):
    t1, t2 = ts(a, b)
    a2, t3 = ts(c, t1)
    return a2, t2 + t3


def vec_sum(xs):
    xs = list(xs)
    n = len(xs)
    e = [0.0] * n
    s = xs[-1]
    for i in range(n - 2, -1, -1):
        s, e[i + 1] = ts(xs[i], s)
    e[0] = s
    return e


def vseb(es, k):
    r = [0.0] * k
    j = 0
    carry = es[0]
    for i in range(1, len(es)):
        s, t = qts(carry, es[i])
        if t != 0.0:
            r[j] = s
            j += 1
            carry = t
            if j == k:
                return r
        else:
            carry = s
    r[j] = carry
    return r


def renorm4(c0, c1, c2, c3, c4):
    e = [0.0] * 5
    s, e[4] = qts(c3, c4)
    s, e[3] = qts(c2, s)
    s, e[2] = qts(c1, s)
    s, e[1] = qts(c0, s)
    e[0] = s
    r = [0.0] * 4
    j = 0
    carry = 0.0
    for i in range(1, 5):
        if i == 1:
            sv, t = e[0], e[1]
        else:
            sv, t = qts(carry, e[i])
        if t != 0.0:
            r[j] = sv
            j += 1
            carry = t
            if j == 3:
                tail = carry
                for q in range(i + 1, 5):
                    tail = tail + e[q]
                r[3] = tail
                return r
        else:
            carry = sv
    r[j] = carry
    return r


def dd_add(x, y):
    s, e = ts(x[0], y[0])
    e = e + (x[1] + y[1])
    return list(qts(s, e))


def dd_mul(x, y):
    p1, p2 = tp(x[0], y[0])
    p2 = p2 + (x[0] * y[1] + x[1] * y[0])
    return list(qts(p1, p2))


def qd_add(x, y):
    pairs = [ts(a, b) for a, b in zip(x, y)]     # exact sums of the component pairs
    s, t = [p[0] for p in pairs], [p[1] for p in pairs]
    s1, c = ts(s[1], t[0])                        # errors carried one level down
    s2, c, c2 = three_sum(s[2], c, t[1])
    s3, c = three_sum2(s[3], c, t[2])
    return renorm4(s[0], s1, s2, s3, (c + c2) + t[3])


def qd_mul(x, y):
    p0, q0 = tp(x[0], y[0])
    p1, q1 = tp(x[0], y[1])
    p2, q2 = tp(x[1], y[0])
    p3, q3 = tp(x[0], y[2])
    p4, q4 = tp(x[1], y[1])
    p5, q5 = tp(x[2], y[0])
    p1, p2, q0 = three_sum(p1, p2, q0)
    p2, q1, q2 = three_sum(p2, q1, q2)
    p3, p4, p5 = three_sum(p3, p4, p5)
    s0, t0 = ts(p2, p3)
    s1, t1 = ts(q1, p4)
    s2 = q2 + p5
    s1, t0 = ts(s1, t0)
    s2 = s2 + (t0 + t1)
    for term in (x[0] * y[3], x[1] * y[2], x[2] * y[1], x[3] * y[0], q0, q3, q4, q5):
        s1 = s1 + term
    return renorm4(p0, p1, s0, s1, s2)


def td_addq(x, y):
    return qd_add([x[0], x[1], x[2], 0.0], [y[0], y[1], y[2], 0.0])[:3]


def td_mul(x, y):
    z00u, z00l = tp(x[0], y[0])
    z01u, z01l = tp(x[0], y[1])
    z10u, z10l = tp(x[1], y[0])
    b = vec_sum([z00l, z01u, z10u])
    c = fma(x[1], y[1], b[2])
    z31 = fma(x[0], y[2], z10l)
    z32 = fma(x[2], y[0], z01l)
    s3 = c + (z31 + z32)
    e = vec_sum([z00u, b[0], b[1], s3])
    return [e[0]] + vseb(e[1:], 2)


ADD = {2: dd_add, 3: td_addq, 4: qd_add}
MUL = {2: dd_mul, 3: td_mul, 4: qd_mul}


# ---------------------------------------------------------------------------
# Evaluation orders, transcribed from their definitions (not from the C
# oracle): the canonical GEMM of eqn (1), Sec. 3 (one ascending chain per
# entry, then the BLAS epilogue), the fixed 64-ary dot tree (Sec. 4) and
# Strassen's seven-product level (Sec. 3, Fig. 5).  Matrices are numpy
# arrays of component planes, shape (P, columns, ld), column-major.

def _entry(X, trans, r, c):
    """Element (r, c) of op(X) as a list of P floats."""
    return [float(v) for v in (X[:, r, c] if trans else X[:, c, r])]


def _is_zero(v):
    return all(x == 0.0 for x in v)


def _is_one(v):
    return v[0] == 1.0 and all(x == 0.0 for x in v[1:])


def _epilogue(P, alpha, acc, beta, c_old, alpha_gone):
    """alpha acc + beta c_old with C never read when beta == 0; alpha == 0 (or
    k == 0) leaves beta c_old, or zero."""
    mul, add = MUL[P], ADD[P]
    if alpha_gone:
        return [0.0] * P if _is_zero(beta) else mul(beta, c_old)
    t = mul(alpha, acc)
    return t if _is_zero(beta) else add(t, mul(beta, c_old))


def gemm(P, ta, tb, m, n, k, alpha, A, B, beta, C):
    """C = alpha op(A) op(B) + beta C, every entry from acc = 0 and
    acc = ADD(acc, MUL(op(A)_il, op(B)_lj)) for l = 0, 1, ..., k-1."""
    import numpy as np
    add, mul = ADD[P], MUL[P]
    alpha = [float(v) for v in alpha][:P]
    beta = [float(v) for v in beta][:P]
    out = np.array(C, dtype=np.float64, copy=True)
    gone = k == 0 or _is_zero(alpha)
    if m == 0 or n == 0 or (gone and _is_one(beta)):
        return out
    at, bt = ta in "TtCc", tb in "TtCc"
    for j in range(n):
        for i in range(m):
            acc = [0.0] * P
            if not gone:
                for l in range(k):
                    acc = add(acc, mul(_entry(A, at, i, l), _entry(B, bt, l, j)))
            out[:, j, i] = _epilogue(P, alpha, acc, beta, [float(v) for v in out[:, j, i]], gone)
    return out


def dot(P, x, y, fanin=64):
    """sum_i x_i y_i: products summed from zero in ascending order within
    blocks of `fanin` consecutive terms, then the block sums the same way in
    blocks of `fanin`, level after level, until one value is left."""
    add, mul = ADD[P], MUL[P]
    n = x.shape[1]
    if n == 0:
        return [0.0] * P
    vals = []
    for b0 in range(0, n, fanin):
        acc = [0.0] * P
        for i in range(b0, min(n, b0 + fanin)):
            acc = add(acc, mul([float(v) for v in x[:, i]], [float(v) for v in y[:, i]]))
        vals.append(acc)
    while len(vals) > 1:
        nxt = []
        for b0 in range(0, len(vals), fanin):
            acc = [0.0] * P
            for v in vals[b0:b0 + fanin]:
                acc = add(acc, v)
            nxt.append(acc)
        vals = nxt
    return vals[0]


def _op_dense(X, trans, rows, cols):
    """op(X) as a rows x cols list of lists of P-lists."""
    return [[_entry(X, trans, r, c) for c in range(cols)] for r in range(rows)]


def _blk(M, bi, bj, h, w):
    return [row[bj * w:(bj + 1) * w] for row in M[bi * h:(bi + 1) * h]]


def _plus(P, X, Y, sign=1):
    """X + Y (sign 1) or X + (-Y) (sign -1, exact negation), entry by entry."""
    add = ADD[P]
    return [[add(x, y if sign > 0 else [-v for v in y]) for x, y in zip(rx, ry)]
            for rx, ry in zip(X, Y)]


def _product(P, X, Y, levels):
    """X (h x q) times Y (q x w): Strassen's seven products for `levels`
    levels, canonical-order block products (alpha 1, beta 0) below."""
    import numpy as np
    h, q, w = len(X), len(Y), len(Y[0]) if Y else 0
    if levels == 0:
        A = np.zeros((P, q, max(h, 1)))
        B = np.zeros((P, w, max(q, 1)))
        for r in range(h):
            for c in range(q):
                A[:, c, r] = X[r][c]
        for r in range(q):
            for c in range(w):
                B[:, c, r] = Y[r][c]
        one = [1.0] + [0.0] * (P - 1)
        Cb = gemm(P, "N", "N", h, w, q, one, A, B, [0.0] * P, np.zeros((P, w, max(h, 1))))
        return [[[float(v) for v in Cb[:, c, r]] for c in range(w)] for r in range(h)]
    a, c, b = h // 2, q // 2, w // 2
    A11, A12, A21, A22 = (_blk(X, i, j, a, c) for i, j in ((0, 0), (0, 1), (1, 0), (1, 1)))
    B11, B12, B21, B22 = (_blk(Y, i, j, c, b) for i, j in ((0, 0), (0, 1), (1, 0), (1, 1)))
    L = levels - 1
    M1 = _product(P, _plus(P, A11, A22), _plus(P, B11, B22), L)
    M2 = _product(P, _plus(P, A21, A22), B11, L)
    M3 = _product(P, A11, _plus(P, B12, B22, -1), L)
    M4 = _product(P, A22, _plus(P, B21, B11, -1), L)
    M5 = _product(P, _plus(P, A11, A12), B22, L)
    M6 = _product(P, _plus(P, A21, A11, -1), _plus(P, B11, B12), L)
    M7 = _product(P, _plus(P, A12, A22, -1), _plus(P, B21, B22), L)
    C11 = _plus(P, _plus(P, _plus(P, M1, M4), M5, -1), M7)
    C12 = _plus(P, M3, M5)
    C21 = _plus(P, M2, M4)
    C22 = _plus(P, _plus(P, _plus(P, M1, M2, -1), M3), M6)
    top = [r1 + r2 for r1, r2 in zip(C11, C12)]
    bottom = [r1 + r2 for r1, r2 in zip(C21, C22)]
    return top + bottom


def gemm_strassen(P, levels, ta, tb, m, n, k, alpha, A, B, beta, C):
    """C = alpha op(A) op(B) + beta C with the product from `levels` levels of
    Strassen's method, then the canonical epilogue."""
    import numpy as np
    alpha = [float(v) for v in alpha][:P]
    beta = [float(v) for v in beta][:P]
    out = np.array(C, dtype=np.float64, copy=True)
    gone = k == 0 or _is_zero(alpha)
    if m == 0 or n == 0 or (gone and _is_one(beta)):
        return out
    prod = None if gone else _product(P, _op_dense(A, ta in "TtCc", m, k), _op_dense(B, tb in "TtCc", k, n),
                                      levels)
    for j in range(n):
        for i in range(m):
            acc = [0.0] * P if gone else prod[i][j]
            out[:, j, i] = _epilogue(P, alpha, acc, beta, [float(v) for v in out[:, j, i]], gone)
    return out
