"""Exact arithmetic for checking results: every binary64 is an exact dyadic
rational, so sums and products of them are evaluated here with Python's
unbounded integers (no rounding anywhere).

Used to pin the oracle (EFT invariants, error bounds against the exact
product) and to measure the error of GPU results on sampled entries.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

UNIT = {2: Fraction(1, 2 ** 104), 3: Fraction(1, 2 ** 150), 4: Fraction(1, 2 ** 200)}


def frac(x: float) -> Fraction:
    return Fraction(float(x))


def mp_frac(comps) -> Fraction:
    """Exact value of a multi-component number (sum of its components)."""
    return sum((Fraction(float(c)) for c in comps), Fraction(0))


def _dyadic(x: np.ndarray):
    """Integer mantissas and exponents with x == m * 2**e exactly (m, e int64)."""
    f, e = np.frexp(x)
    m = np.ldexp(f, 53).astype(np.int64)      # exact: f has 53 significant bits
    return m, e.astype(np.int64) - 53


def to_scaled_ints(planes: np.ndarray):
    """Exact values of a list of multi-component numbers as integers over a
    common power of two.  planes: (P, N).  Returns (list of N Python ints, Z)
    with value_t == ints[t] * 2**-Z exactly."""
    P, N = planes.shape
    m, e = _dyadic(planes.reshape(-1))
    nz = m != 0
    Z = int(-e[nz].min()) if nz.any() else 0
    out = [0] * N
    mm = m.reshape(P, N)
    ee = e.reshape(P, N)
    for c in range(P):
        for t in range(N):
            mv = int(mm[c, t])
            if mv:
                out[t] += mv << int(ee[c, t] + Z)
    return out, Z


def exact_dot(a_planes: np.ndarray, b_planes: np.ndarray) -> Fraction:
    """Exact sum_l a_l * b_l for multi-component vectors a, b of shape (P, k)."""
    ai, za = to_scaled_ints(a_planes)
    bi, zb = to_scaled_ints(b_planes)
    s = sum(x * y for x, y in zip(ai, bi))
    return Fraction(s, 1 << (za + zb))


def abs_dot(a_planes: np.ndarray, b_planes: np.ndarray) -> Fraction:
    """Exact sum_l |a_l| * |b_l|."""
    ai, za = to_scaled_ints(a_planes)
    bi, zb = to_scaled_ints(b_planes)
    s = sum(abs(x) * abs(y) for x, y in zip(ai, bi))
    return Fraction(s, 1 << (za + zb))


def op_row(A: np.ndarray, trans: str, i: int, k: int) -> np.ndarray:
    """Row i of op(A) as (P, k); A in component planes (P, cols, ld)."""
    if trans in "Nn":
        return A[:, :k, i]
    return A[:, i, :k]


def op_col(B: np.ndarray, trans: str, j: int, k: int) -> np.ndarray:
    """Column j of op(B) as (P, k)."""
    if trans in "Nn":
        return B[:, j, :k]
    return B[:, :k, j]


class GemmChecker:
    """Exact C* = alpha op(A) op(B) + beta C0 on sampled entries, and the
    error of a computed C relative to k*u*(|alpha||A||B| + |beta||C0|)."""

    def __init__(self, P, ta, tb, m, n, k, alpha, A, B, beta, C0):
        self.P, self.ta, self.tb, self.m, self.n, self.k = P, ta, tb, m, n, k
        self.alpha = mp_frac(alpha)
        self.beta = mp_frac(beta)
        self.A, self.B, self.C0 = A, B, C0
        self._rows, self._cols = {}, {}

    def _row(self, i):
        if i not in self._rows:
            self._rows[i] = to_scaled_ints(np.ascontiguousarray(op_row(self.A, self.ta, i, self.k)))
        return self._rows[i]

    def _col(self, j):
        if j not in self._cols:
            self._cols[j] = to_scaled_ints(np.ascontiguousarray(op_col(self.B, self.tb, j, self.k)))
        return self._cols[j]

    def entry(self, i, j):
        """(exact value, bound base) for entry (i, j); computed once per entry."""
        memo = self.__dict__.setdefault("_entries", {})
        if (i, j) not in memo:
            memo[(i, j)] = self._entry(i, j)
        return memo[(i, j)]

    def _entry(self, i, j):
        if self.k > 0:
            ai, za = self._row(i)
            bj, zb = self._col(j)
            dot = Fraction(sum(x * y for x, y in zip(ai, bj)), 1 << (za + zb))
            adot = Fraction(sum(abs(x) * abs(y) for x, y in zip(ai, bj)), 1 << (za + zb))
        else:
            dot = adot = Fraction(0)
        exact = self.alpha * dot
        base = abs(self.alpha) * adot
        if self.beta != 0:
            c0 = mp_frac(self.C0[:, j, i])
            exact += self.beta * c0
            base += abs(self.beta) * abs(c0)
        return exact, base

    def ratios(self, C, entries):
        """err / (max(k,1) * u * base) for each (i, j) in entries."""
        u = UNIT[self.P]
        out = []
        for i, j in entries:
            exact, base = self.entry(i, j)
            got = mp_frac(C[:, j, i])
            err = abs(got - exact)
            if base == 0:
                out.append(0.0 if err == 0 else float("inf"))
            else:
                out.append(float(err / (max(self.k, 1) * u * base)))
        return np.array(out)


def sample_entries(rng, m, n, count=1024):
    """Grid sample: ~sqrt(count) distinct rows x ~sqrt(count) distinct columns."""
    r = max(1, min(m, int(round(count ** 0.5))))
    c = max(1, min(n, count // r))
    rows = np.sort(rng.choice(m, size=r, replace=False))
    cols = np.sort(rng.choice(n, size=c, replace=False))
    return [(int(i), int(j)) for i in rows for j in cols]
