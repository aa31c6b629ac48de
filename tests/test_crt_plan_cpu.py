"""The residue form's modulus count (host logic, no GPU) against its
definition in exact integers.  Digits are signed 7-bit, so the largest digit
integer of d digits is a(d) = 64 (128^d - 1) / 127 and |C'| <= k a(s)^2; the
residues modulo M determine C' when M > 2 k a(s)^2.  The moduli are the
greedy pairwise coprime ones from 256 down.  With two levels (QD, 25 <= s <=
32) the largest of the three half-size products is ss, bounded by k (a(hi) +
a(lo))^2 with hi = ceil(s/2), lo = floor(s/2), and at most 33 moduli are
used.  The library takes the count from logarithms with a 0.01-bit margin, so
it may take one modulus more than the least, only where the least one's
product is within that margin of the bound."""
import math

import pytest

import paper_2101_06584_amd as mp

def greedy_moduli(count=49):
    out = []
    for m in range(256, 1, -1):
        if all(math.gcd(m, q) == 1 for q in out):
            out.append(m)
        if len(out) == count:
            break
    return out


MODULI = greedy_moduli()
PREFIX = [math.prod(MODULI[:N]) for N in range(50)]


def amax(d):
    return 64 * (128 ** d - 1) // 127


def least(bound, cap):
    """Smallest N <= cap with M_N > bound, else 0."""
    return next((N for N in range(1, cap + 1) if PREFIX[N] > bound), 0)


def within_margin(N, bound):
    return N > 0 and PREFIX[N] <= bound * 2 ** 0.01


def check(got, bound, cap):
    N = least(bound, cap)
    if N == 0:
        # none suffices; the margin could only make the library refuse more
        assert got == 0
        return 0
    if got == 0:
        # the margin pushed the count past the cap
        assert N == cap and within_margin(N, bound), (got, N)
    else:
        assert got >= N, (got, N)                     # enough moduli, always
        assert got == N or (got == N + 1 and within_margin(N, bound)), (got, N)
    return got


def test_moduli_are_pairwise_coprime_and_bounded():
    assert len(MODULI) == 49 and MODULI[0] == 256 and MODULI[-1] == 29
    assert all(math.gcd(a, b) == 1 for i, a in enumerate(MODULI) for b in MODULI[i + 1:])
    assert 341 < math.log2(PREFIX[49]) < 342


KS = [1, 2, 3, 31, 32, 33, 63, 64, 100, 114, 115, 127, 1000, 4096, 8192, 8193, 65535, 65536, 131071]


@pytest.mark.parametrize("P", [2, 3, 4])
def test_modulus_count_matches_definition(P):
    for s in range(1, 35):
        for k in KS:
            got = mp.crt_moduli(P, k, s)
            if s <= 24:
                # one level for every precision (QD too: no second level below 25 digits)
                check(got, 2 * k * amax(s) ** 2, 49)
            elif P != 4 or s > 32:
                assert got == 0, (P, k, s, got)
            else:
                hi, lo = (s + 1) // 2, s // 2
                assert got % 3 == 0, (k, s, got)
                check(got // 3, 2 * k * (amax(hi) + amax(lo)) ** 2, 33)


def test_largest_inner_dimension_at_24_digits():
    # one level, s = 24: all 49 moduli hold k a(24)^2 up to k = 115, by less
    # than the margin at 115, so the library stops at 114
    assert PREFIX[49] > 2 * 115 * amax(24) ** 2 and PREFIX[49] <= 2 * 116 * amax(24) ** 2
    assert within_margin(49, 2 * 115 * amax(24) ** 2)
    assert mp.crt_moduli(2, 114, 24) == 49 == mp.crt_moduli(3, 114, 24)
    assert mp.crt_moduli(2, 115, 24) == 0 == mp.crt_moduli(3, 115, 24) == mp.crt_moduli(4, 115, 24)


def test_outside_the_range():
    for P in (2, 3, 4):
        assert mp.crt_moduli(P, 0, 16) == 0 and mp.crt_moduli(P, 131072, 16) == 0
        assert mp.crt_moduli(P, 100, 33) == 0
