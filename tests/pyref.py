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
    s = [x[i] + y[i] for i in range(4)]
    v = [s[i] - x[i] for i in range(4)]
    u = [s[i] - v[i] for i in range(4)]
    w = [x[i] - u[i] for i in range(4)]
    u = [y[i] - v[i] for i in range(4)]
    t = [w[i] + u[i] for i in range(4)]
    s1, t0 = ts(s[1], t[0])
    s2, t0, t1 = three_sum(s[2], t0, t[1])
    s3, t0 = three_sum2(s[3], t0, t[2])
    t0 = (t0 + t1) + t[3]
    return renorm4(s[0], s1, s2, s3, t0)


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
