"""The seeded input generator: deterministic, non-overlapping expansions,
column-major component planes, exact exponent scaling."""
import numpy as np

from tests import synth


def test_deterministic_and_layout():
    a = synth.mp_matrix(1, "A", 3, 7, 5, ld=9)
    b = synth.mp_matrix(1, "A", 3, 7, 5, ld=9)
    assert a.shape == (3, 5, 9) and np.array_equal(a, b)
    assert np.all(a[:, :, 7:] == 0)                     # ld padding untouched
    assert np.abs(a[0]).max() <= 1.0
    assert synth.seed_for(2, "B") == synth.SEED_BASE + 33


def test_components_non_overlapping():
    for P in (2, 3, 4):
        x = synth.mp_matrix(2, "B", P, 64, 64)
        for c in range(1, P):
            assert np.all(np.abs(x[c]) < 0.5 * np.spacing(np.abs(x[c - 1])))
            # adding the lower part to the upper one leaves it unchanged
            assert np.array_equal(x[c - 1] + x[c], x[c - 1])


def test_exponent_spread_is_exact_power_of_two_scaling():
    base = synth.mp_matrix(3, "A", 4, 16, 16)
    spread = synth.mp_matrix(3, "A", 4, 16, 16, exp_range=(-30, 30))
    ratio = spread / base
    e = np.log2(np.abs(ratio[0]))
    assert np.array_equal(e, np.round(e)) and e.min() >= -30 and e.max() <= 30
    assert np.array_equal(ratio[0], ratio[3])


def test_paper_matrices_components():
    A, B = synth.paper_matrices(5, 2)
    # A[i, j] = sqrt5 (i + j - 1): symmetric in i, j
    assert np.array_equal(A[:, 2, 1], A[:, 1, 2])
    assert abs(A[0, 0, 0] - 5 ** 0.5) < 1e-15
    assert np.all(B[:, :, 4] == 0)                      # row i = n: sqrt3 * 0
