"""Seeded synthetic inputs for DD/TD/QD matrices, shared by the oracle tests,
the GPU tests and the benchmark.

This module only draws random numbers and lays them out; it performs none of
the multi-component arithmetic under test (no TwoSum, no renormalisation).

Storage convention ("component planes", the structure-of-arrays layout of
Sec. 2.5 / Fig. 1): a P-component matrix with `rows` x `cols` entries is a
float64 array of shape (P, cols, ld), ld >= rows.  Plane c holds component c
(c = 0 most significant) of every entry in column-major order, so entry
(i, j) of component c is arr[c, j, i].  The plane stride is cols * ld.

Value distribution (the workloads of the benchmark section, Sec. 3, made
random): component 0 is uniform in [-1, 1]; each further component is
uniform in (-ulp/2, +ulp/2) of the component before it, i.e. the expansion
is non-overlapping by construction and needs no renormalisation pass.
"""
from __future__ import annotations

from fractions import Fraction
import math

import numpy as np

SEED_BASE = 2101065840
SLOT = {"A": 0, "B": 1, "C": 2, "alpha": 3, "beta": 4, "expA": 5, "expB": 6,
        "samples": 7, "shapes": 8}
PREC_P = {"dd": 2, "td": 3, "qd": 4}


def seed_for(family: int, slot: str | int) -> int:
    """Seed of one input (slot) of one family; each workload draws from its
    own family (2: the square benchmark step, 3: QD n = 2048 with exponent
    spread, 4: DD n = 8192, 5: the batched sets; others: tests)."""
    s = SLOT[slot] if isinstance(slot, str) else int(slot)
    return SEED_BASE + 16 * int(family) + s


def rng_for(family: int, slot: str | int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(family, slot)))


def _tail_components(rng, lead: np.ndarray, P: int) -> np.ndarray:
    out = np.empty((P,) + lead.shape, dtype=np.float64)
    out[0] = lead
    for c in range(1, P):
        # half an ulp of a normal x = f 2^e (f in [1/2, 1)) is 2^(e - 54);
        # components here are never subnormal, and a zero gets a zero tail
        prev = out[c - 1]
        _, e = np.frexp(prev)
        half_ulp = np.where(prev == 0.0, 0.0, np.ldexp(1.0, e - 54))
        v = rng.uniform(-1.0, 1.0, size=lead.shape)
        out[c] = half_ulp * v          # |v| < 1 keeps |out[c]| < ulp/2
    return out


def mp_uniform(rng, P: int, shape) -> np.ndarray:
    """P-component numbers, leading part uniform in [-1, 1]; shape (P, *shape)."""
    lead = rng.uniform(-1.0, 1.0, size=shape)
    return _tail_components(rng, lead, P)


def mp_matrix(family: int, slot: str, P: int, rows: int, cols: int, ld: int | None = None,
              exp_range: tuple[int, int] | None = None, exp_mode: str = "entry") -> np.ndarray:
    """A (P, cols, ld) component-plane matrix.

    exp_range=(lo, hi) multiplies every entry exactly by 2**e with e drawn
    uniformly from the integers lo..hi: per entry (exp_mode="entry"), or one e
    per row ("row") or per column ("col").
    """
    ld = rows if ld is None else ld
    assert ld >= max(1, rows)
    rng = rng_for(family, slot)
    core = mp_uniform(rng, P, (cols, rows))          # column-major: [j][i]
    if exp_range is not None:
        erng = rng_for(family, "expA" if slot == "A" else "expB" if slot == "B" else 9)
        lo, hi = exp_range
        if exp_mode == "entry":
            e = erng.integers(lo, hi + 1, size=(cols, rows))
        elif exp_mode == "row":
            e = np.broadcast_to(erng.integers(lo, hi + 1, size=(1, rows)), (cols, rows))
        elif exp_mode == "col":
            e = np.broadcast_to(erng.integers(lo, hi + 1, size=(cols, 1)), (cols, rows))
        else:
            raise ValueError(exp_mode)
        core = np.ldexp(core, e[None, :, :].astype(np.int32))
    out = np.zeros((P, cols, ld), dtype=np.float64)
    out[:, :, :rows] = core
    return out


def mp_scalar(family: int, slot: str, P: int) -> np.ndarray:
    rng = rng_for(family, slot)
    return mp_uniform(rng, P, (1,))[:, 0].copy()


def mp_one(P: int) -> np.ndarray:
    v = np.zeros(P)
    v[0] = 1.0
    return v


def mp_vector(seed: int, P: int, n: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return mp_uniform(rng, P, (n,))


# ---------------------------------------------------------------------------
# The fixed test matrices of the benchmark section (Sec. 3):
#   A = [sqrt(5) (i + j - 1)],  B = [sqrt(3) (n - i)],  i, j = 1..n
# Each entry is rounded to a P-component expansion by repeated round-to-nearest
# of the exact remainder (Python's int/int true division is correctly rounded).
# ---------------------------------------------------------------------------
def sqrt_fraction(v: int, bits: int = 700) -> Fraction:
    """sqrt(v) to within 2**-bits (floor), as an exact rational."""
    return Fraction(math.isqrt(v << (2 * bits)), 1 << bits)


def fraction_to_components(x: Fraction, P: int) -> list[float]:
    comps = []
    r = x
    for _ in range(P):
        c = float(r)                 # correctly rounded
        comps.append(c)
        r = r - Fraction(c)
    return comps


def paper_matrices(n: int, P: int):
    """Column-major component planes (P, n, n) of the paper's A and B."""
    r5 = sqrt_fraction(5)
    r3 = sqrt_fraction(3)
    a_vals = {t: fraction_to_components(r5 * t, P) for t in range(1, 2 * n)}
    b_vals = {t: fraction_to_components(r3 * t, P) for t in range(0, n)}
    A = np.zeros((P, n, n))
    B = np.zeros((P, n, n))
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            A[:, j - 1, i - 1] = a_vals[i + j - 1]
            B[:, j - 1, i - 1] = b_vals[n - i]
    return A, B


def paper_exact_entry(n: int, i: int) -> Fraction:
    """Exact c_ij of the paper's product (independent of j), 1-based i:
    sum_k sqrt5 (i+k-1) sqrt3 (n-k) = sqrt15 * n(n-1)(3i+n-2)/6."""
    r15 = sqrt_fraction(15)
    return r15 * Fraction(n * (n - 1) * (3 * i + n - 2), 6)


def batch_problems(family: int, P: int, count: int, lo: int, hi: int):
    """`count` GEMM problems with m, n, k drawn uniformly from lo..hi (slot
    "shapes"); operands drawn like mp_matrix in one pass (slots A, B, C) and
    cut per problem.  alpha = 1, beta = 0 (C = A B), transposes 'N'."""
    shapes = rng_for(family, "shapes").integers(lo, hi + 1, size=(count, 3))
    sizes = [(int(m) * int(k), int(k) * int(n), int(m) * int(n)) for m, n, k in shapes]
    pools = {}
    for slot, idx in (("A", 0), ("B", 1), ("C", 2)):
        total = sum(s[idx] for s in sizes)
        rows = (total + 1023) // 1024            # drawn as rows of 1024 (faster in numpy)
        pools[slot] = mp_uniform(rng_for(family, slot), P, (rows, 1024)).reshape(P, -1)[:, :total]
    off = [0, 0, 0]
    out = []
    for (m, n, k), sz in zip(shapes, sizes):
        m, n, k = int(m), int(n), int(k)
        mats = []
        for idx, (slot, rows, cols) in enumerate((("A", m, k), ("B", k, n), ("C", m, n))):
            flat = pools[slot][:, off[idx]:off[idx] + sz[idx]]
            off[idx] += sz[idx]
            mats.append(np.ascontiguousarray(flat.reshape(P, cols, rows)))
        out.append(dict(transa="N", transb="N", m=m, n=n, k=k, A=mats[0], B=mats[1], C=mats[2],
                        alpha=mp_one(P), beta=np.zeros(P)))
    return out
