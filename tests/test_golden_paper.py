"""The fixed test matrices of the paper's benchmark section (Sec. 3),
stored in tests/golden/paper_matrices.txt as integer coefficients of sqrt5,
sqrt3 and sqrt15 (written by tests/golden/make_paper_matrices.py with exact
integer arithmetic).  Pins the fixture to its definition and to the closed
form of the product, the test generator's rounding of A and B to the
fixture, and the oracle's product to the paper's statement that these
matrices lose at most one or two decimal digits."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import synth

HERE = os.path.dirname(os.path.abspath(__file__))
U = {2: Fraction(1, 2 ** 104), 3: Fraction(1, 2 ** 150), 4: Fraction(1, 2 ** 200)}


def fixture():
    out, cur = {}, None
    with open(os.path.join(HERE, "golden", "paper_matrices.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, *vals = line.split()
            if head == "n":
                cur = int(vals[0])
                out[cur] = {"A": [], "B": [], "C": []}
            else:
                out[cur][head].append([int(v) for v in vals])
    return out


GOLD = fixture()


def frac(comps):
    return sum((Fraction(float(c)) for c in comps), Fraction(0))


def test_fixture_matches_its_definition():
    assert sorted(GOLD) == [1, 2, 4, 7, 32]
    for n, g in GOLD.items():
        assert all(len(g[x]) == n and all(len(r) == n for r in g[x]) for x in "ABC")
        for i in range(1, n + 1):
            for j in range(1, n + 1):
                assert g["A"][i - 1][j - 1] == i + j - 1
                assert g["B"][i - 1][j - 1] == n - i
                # brute force over l, and the closed form n (n - 1)(3 i + n - 2) / 6
                assert g["C"][i - 1][j - 1] == sum((i + l - 1) * (n - l) for l in range(1, n + 1))
                assert 6 * g["C"][i - 1][j - 1] == n * (n - 1) * (3 * i + n - 2)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_generator_rounds_the_fixture(P):
    r5, r3 = synth.sqrt_fraction(5), synth.sqrt_fraction(3)
    for n in (4, 7):
        A, B = synth.paper_matrices(n, P)
        for i in range(n):
            for j in range(n):
                for M, r, coef in ((A, r5, GOLD[n]["A"][i][j]), (B, r3, GOLD[n]["B"][i][j])):
                    x = r * coef
                    # P components, each rounded to nearest: within 2^-(53 P) |x|
                    assert abs(frac(M[:, j, i]) - x) <= x / 2 ** (53 * P - 1)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_oracle_loses_at_most_two_digits(P):
    r15 = synth.sqrt_fraction(15)
    one, zero = synth.mp_one(P), np.zeros(P)
    for n in (1, 2, 4, 7, 32):
        A, B = synth.paper_matrices(n, P)
        C = oracle.gemm(P, "N", "N", n, n, n, one, A, B, zero, np.zeros((P, n, n)))
        for i in range(n):
            for j in range(n):
                c = GOLD[n]["C"][i][j]
                got = frac(C[:, j, i])
                if c == 0:
                    assert got == 0
                    continue
                exact = r15 * c
                assert synth.paper_exact_entry(n, i + 1) == exact
                rel = abs(got - exact) / exact
                assert rel <= 100 * U[P], (P, n, i, j, float(rel))
