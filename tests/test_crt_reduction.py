"""The residue form's reduction of an INT8 product's int32 sums: q =
floor(fma(x, 1/m, 2^-20)) with 1/m rounded to binary64, then x - q m, gives
x mod m in [0, m) for every |x| < 2^31 and every modulus m <= 256.

fma is modelled exactly (the exact value x * inv + 2^-20, then one rounding
to binary64, via Python's correctly rounded Fraction-to-float); the cases
are the ones the argument turns on: exact multiples of m and their
neighbours (one above, one below, m / 2 above), near zero and at both ends
of the int32 range, for every m from 2 to 256 (a superset of the moduli)."""
import math
import random
from fractions import Fraction


def fma_binary64(x, inv, c):
    return float(Fraction(x) * Fraction(inv) + Fraction(c))


def reduce_mod(x, m):
    q = math.floor(fma_binary64(x, 1.0 / m, 2.0 ** -20))
    return x - q * m          # the kernel's fma(-q, m, x): an integer below 2^53, exact


def test_reduction_is_exact_at_multiples_and_neighbours():
    rng = random.Random(20260)
    lo, hi = -(2 ** 31), 2 ** 31
    for m in range(2, 257):
        top = hi // m
        js = {0, 1, -1, top, -top, top - 1, -top - 1}
        js.update(rng.randrange(-top, top) for _ in range(10))
        for j in js:
            for d in (-1, 0, 1, m // 2, m - 1):
                x = j * m + d
                if lo <= x < hi:
                    assert reduce_mod(x, m) == x % m, (m, x)
    for x in (lo, hi - 1):
        for m in (3, 251, 256):
            assert reduce_mod(x, m) == x % m
