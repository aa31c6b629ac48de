"""Host-side argument checks of the plain entry points under random calls
(CPU, no GPU work): a valid random call with one or two arguments made
invalid returns -(position of the first invalid argument), whatever the
precision, shape, transposes and leading-dimension slack."""
import ctypes as C

import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import paper_2101_06584_amd as mp  # noqa: E402

FAKE = {"A": 0x100000000, "B": 0x200000000, "C": 0x300000000}   # disjoint, never dereferenced
TRANS = "NnTtCc"


def rows_cols(t, r, c):
    """Rows and columns of a stored operand whose op is r x c."""
    return (r, c) if t in "Nn" else (c, r)


@st.composite
def calls(draw):
    P = draw(st.sampled_from([2, 3, 4]))
    ta, tb = draw(st.sampled_from(TRANS)), draw(st.sampled_from(TRANS))
    m, n, k = (draw(st.integers(1, 300)) for _ in range(3))
    ra, ca = rows_cols(ta, m, k)
    rb, cb = rows_cols(tb, k, n)
    lda, ldb, ldc = (r + draw(st.integers(0, 5)) for r in (ra, rb, m))
    a = dict(ta=ta.encode(), tb=tb.encode(), m=m, n=n, k=k, alpha=True, A=FAKE["A"], lda=lda,
             sa=lda * ca + draw(st.integers(0, 9)), B=FAKE["B"], ldb=ldb, sb=ldb * cb + draw(st.integers(0, 9)),
             beta=True, C=FAKE["C"], ldc=ldc, sc=ldc * n + draw(st.integers(0, 9)))
    bad = sorted(set(draw(st.lists(st.integers(1, 16), min_size=1, max_size=2))))
    cut = draw(st.integers(1, 3))
    for i in bad:
        if i == 1: a["ta"] = b"X"
        elif i == 2: a["tb"] = b"Q"
        elif i == 3: a["m"] = -cut
        elif i == 4: a["n"] = -cut
        elif i == 5: a["k"] = -cut
        elif i == 6: a["alpha"] = None
        elif i == 7: a["A"] = None                      # read: alpha != 0 and m, n, k > 0
        elif i == 8: a["lda"] = max(1, ra) - cut
        elif i == 9: a["sa"] = a["lda"] * ca - cut
        elif i == 10: a["B"] = None
        elif i == 11: a["ldb"] = max(1, rb) - cut
        elif i == 12: a["sb"] = a["ldb"] * cb - cut
        elif i == 13: a["beta"] = None
        elif i == 14: a["C"] = None
        elif i == 15: a["ldc"] = max(1, m) - cut
        elif i == 16: a["sc"] = a["ldc"] * n - cut
    return P, a, bad[0]


@settings(max_examples=400, deadline=None)
@given(calls())
def test_first_invalid_argument_is_reported(call):
    P, a, first = call
    L = mp.load()
    fn = {2: L.mpgemm_dd, 3: L.mpgemm_td, 4: L.mpgemm_qd}[P]
    arr = C.c_double * P
    alpha = arr(*([1.0] + [0.0] * (P - 1))) if a["alpha"] else None
    beta = arr(*([0.5] + [0.0] * (P - 1))) if a["beta"] else None
    ptr = lambda v: None if v is None else C.c_void_p(v)
    rc = fn(a["ta"], a["tb"], a["m"], a["n"], a["k"], alpha, ptr(a["A"]), a["lda"], a["sa"], ptr(a["B"]),
            a["ldb"], a["sb"], beta, ptr(a["C"]), a["ldc"], a["sc"], None)
    assert rc == -first, (P, a, first, rc)
