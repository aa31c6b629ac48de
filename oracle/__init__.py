"""ctypes binding of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
load this package.  Arrays are numpy float64 component planes (see
tests/synth.py for the layout).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_i64, _int, _ch = C.c_int64, C.c_int, C.c_char
_dp = C.POINTER(C.c_double)


def lib():
    global _LIB
    if _LIB is None:
        # MPREF_LIB=san selects the sanitizer build (oracle/build.py --sanitize)
        san = os.environ.get("MPREF_LIB") == "san"
        path = os.path.join(_HERE, "libmpref_san.so" if san else "libmpref.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build(sanitize=san)
        L = C.CDLL(path)
        L.ref_vec.argtypes = [_int, _int, _i64, C.c_void_p, _i64, C.c_void_p, _i64, C.c_void_p, _i64]
        L.ref_vec.restype = _int
        L.ref_prim.argtypes = [_int, _i64, C.c_void_p, C.c_void_p]
        L.ref_prim.restype = _int
        L.ref_gemm.argtypes = [_int, _ch, _ch, _i64, _i64, _i64, C.c_void_p, C.c_void_p, _i64, _i64,
                               C.c_void_p, _i64, _i64, C.c_void_p, C.c_void_p, _i64, _i64, _i64, _i64,
                               _i64, _i64, _int]
        L.ref_gemm.restype = _int
        L.ref_gemm_v.argtypes = [_int, _int] + L.ref_gemm.argtypes[1:]
        L.ref_gemm_v.restype = _int
        L.ref_gemm_strassen.argtypes = [_int, _int, _ch, _ch, _i64, _i64, _i64, C.c_void_p, C.c_void_p,
                                        _i64, _i64, C.c_void_p, _i64, _i64, C.c_void_p, C.c_void_p,
                                        _i64, _i64]
        L.ref_gemm_strassen.restype = _int
        L.ref_gemm_crt.argtypes = [_int, _int, _ch, _ch, _i64, _i64, _i64, C.c_void_p, C.c_void_p, _i64,
                                   _i64, C.c_void_p, _i64, _i64, C.c_void_p, C.c_void_p, _i64, _i64,
                                   _i64, _i64, _i64, _i64, _int]
        L.ref_gemm_crt.restype = _int
        L.ref_axpy.argtypes = [_int, _i64, C.c_void_p, C.c_void_p, _i64, C.c_void_p, _i64]
        L.ref_axpy.restype = _int
        L.ref_dot.argtypes = [_int, _i64, C.c_void_p, _i64, C.c_void_p, _i64, C.c_void_p]
        L.ref_dot.restype = _int
        L.ref_gemv.argtypes = [_int, _ch, _i64, _i64, C.c_void_p, C.c_void_p, _i64, _i64, C.c_void_p, _i64,
                               C.c_void_p, C.c_void_p, _i64]
        L.ref_gemv.restype = _int
        L.ref_gemm_split.argtypes = [_int, _int, _ch, _ch, _i64, _i64, _i64, C.c_void_p, C.c_void_p, _i64,
                                     _i64, C.c_void_p, _i64, _i64, C.c_void_p, C.c_void_p, _i64, _i64,
                                     _i64, _i64, _i64, _i64, _int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ref_gemm_split.restype = _int
        L.ref_split_exponents.argtypes = [_int, _ch, _int, _i64, _i64, C.c_void_p, _i64, _i64, C.c_void_p]
        L.ref_split_exponents.restype = None
        L.ref_split_slices.argtypes = [_int, _int, _ch, _int, _i64, _i64, C.c_void_p, _i64, _i64,
                                       C.c_void_p, C.c_void_p]
        L.ref_split_slices.restype = None
        L.ref_split_recombine.argtypes = [_int, _int, _i64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ref_split_recombine.restype = _int
        L.ref_num_threads.restype = _int
        _LIB = L
    return _LIB


def _check_gemm(P, ta, tb, m, n, k, A, B, C):
    """The stored planes must hold op(A) (m x k), op(B) (k x n) and C (m x n):
    (P, cols, ld) with ld >= rows; the C code trusts these sizes."""
    def need(X, name, rows, cols):
        if X.ndim != 3 or X.shape[0] != P:
            raise ValueError(f"{name}: expected (P={P}, cols, ld), got {X.shape}")
        if rows > 0 and cols > 0 and (X.shape[2] < rows or X.shape[1] < cols):
            raise ValueError(f"{name}: {X.shape} cannot hold {rows} x {cols}")
    need(A, "A", *((m, k) if ta in "Nn" else (k, m)))
    need(B, "B", *((k, n) if tb in "Nn" else (n, k)))
    need(C, "C", m, n)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


PRIM = {"quick_two_sum": (0, 2, 2), "two_sum": (1, 2, 2), "two_prod": (2, 2, 2),
        "three_sum": (3, 3, 3), "three_sum2": (4, 3, 2), "vec_sum4": (5, 4, 4),
        "vseb2": (6, 3, 2), "renorm4": (7, 5, 4), "vseb3": (8, 6, 3), "vec_sum3": (9, 3, 3),
        "merge3": (10, 6, 6)}


def prim(name: str, *args):
    """Apply a primitive to equal-length float64 arrays; returns a tuple."""
    which, nin, nout = PRIM[name]
    assert len(args) == nin
    n = len(args[0])
    inp = _f64(np.stack([np.asarray(a, dtype=np.float64) for a in args]))
    out = np.zeros((nout, n))
    rc = lib().ref_prim(which, n, _ptr(inp), _ptr(out))
    assert rc == 0
    return tuple(out[q] for q in range(nout))


VEC_OPS = {"add": 0, "mul": 1, "add_acc": 2, "mulq": 3}


def vec(P: int, op: str, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Element-wise op of (P, n) arrays: "add", "mul", and for TD "add_acc"
    (the accurate addition, Algorithm 3) and "mulq" (TDmulq)."""
    x = _f64(x)
    y = _f64(y)
    n = x.shape[1]
    r = np.zeros_like(x)
    rc = lib().ref_vec(P, VEC_OPS[op], n, _ptr(x), n, _ptr(y), n, _ptr(r), n)
    assert rc == 0, rc
    return r


def gemm(P, ta, tb, m, n, k, alpha, A, B, beta, C, rows=None, cols=None, nthreads=0, variant=0):
    """C = alpha op(A) op(B) + beta C in the canonical order; returns a new C.
    A, B, C are (P, cols, ld) component planes; rows=(r0, r1) / cols=(c0, c1)
    limit the computed block (the rest of C is returned unchanged).  For TD,
    variant bit 0 selects the accurate addition (Algorithm 3), bit 1 TDmulq."""
    A = _f64(A)
    B = _f64(B)
    Cout = _f64(C).copy()
    _check_gemm(P, ta, tb, m, n, k, A, B, Cout)
    alpha = _f64(alpha)
    beta = _f64(beta)
    r0, r1 = rows if rows is not None else (0, -1)
    c0, c1 = cols if cols is not None else (0, -1)
    rc = lib().ref_gemm_v(P, variant, ta.encode(), tb.encode(), m, n, k, _ptr(alpha), _ptr(A),
                          A.shape[2], A.shape[1] * A.shape[2], _ptr(B), B.shape[2],
                          B.shape[1] * B.shape[2], _ptr(beta), _ptr(Cout), Cout.shape[2],
                          Cout.shape[1] * Cout.shape[2], r0, r1, c0, c1, nthreads)
    assert rc == 0, rc
    return Cout


def axpy(P, alpha, x, y):
    """Returns alpha x + y for (P, n) arrays, element by element."""
    x = _f64(x)
    yo = _f64(y).copy()
    n = x.shape[1]
    rc = lib().ref_axpy(P, n, _ptr(_f64(alpha)), _ptr(x), n, _ptr(yo), n)
    assert rc == 0, rc
    return yo


def dot(P, x, y):
    """The dot product of (P, n) arrays in the fixed 64-ary tree order."""
    x = _f64(x)
    y = _f64(y)
    n = x.shape[1]
    r = np.zeros(P)
    rc = lib().ref_dot(P, n, _ptr(x), n, _ptr(y), n, _ptr(r))
    assert rc == 0, rc
    return r


def gemv(P, trans, m, n, alpha, A, x, beta, y):
    """y = alpha op(A) x + beta y; A is (P, n, lda) column-major m x n; x, y are
    (P, len) arrays.  Returns a new y."""
    A = _f64(A)
    x = _f64(x)
    yo = _f64(y).copy()
    rc = lib().ref_gemv(P, trans.encode(), m, n, _ptr(_f64(alpha)), _ptr(A), A.shape[2],
                        A.shape[1] * A.shape[2], _ptr(x), x.shape[1], _ptr(_f64(beta)), _ptr(yo),
                        yo.shape[1])
    assert rc == 0, rc
    return yo


def gemm_strassen(P, levels, ta, tb, m, n, k, alpha, A, B, beta, C):
    """C = alpha op(A) op(B) + beta C with `levels` levels of Strassen's method
    over canonical-order block products; returns a new C (m, n, k must be
    multiples of 2^levels)."""
    A = _f64(A)
    B = _f64(B)
    Cout = _f64(C).copy()
    _check_gemm(P, ta, tb, m, n, k, A, B, Cout)
    alpha = _f64(alpha)
    beta = _f64(beta)
    rc = lib().ref_gemm_strassen(P, levels, ta.encode(), tb.encode(), m, n, k, _ptr(alpha), _ptr(A),
                                 A.shape[2], A.shape[1] * A.shape[2], _ptr(B), B.shape[2],
                                 B.shape[1] * B.shape[2], _ptr(beta), _ptr(Cout), Cout.shape[2],
                                 Cout.shape[1] * Cout.shape[2])
    assert rc == 0, rc
    return Cout


def gemm_crt(P, s, ta, tb, m, n, k, alpha, A, B, beta, C, rows=None, cols=None, nthreads=0):
    """Residue (CRT) form: the exact product of the s-digit integers of the
    split form (full square of digit pairs), rounded to P components; returns
    a new C."""
    A = _f64(A)
    B = _f64(B)
    Cout = _f64(C).copy()
    _check_gemm(P, ta, tb, m, n, k, A, B, Cout)
    alpha = _f64(alpha)
    beta = _f64(beta)
    r0, r1 = rows if rows is not None else (0, -1)
    c0, c1 = cols if cols is not None else (0, -1)
    rc = lib().ref_gemm_crt(P, s, ta.encode(), tb.encode(), m, n, k, _ptr(alpha), _ptr(A), A.shape[2],
                            A.shape[1] * A.shape[2], _ptr(B), B.shape[2], B.shape[1] * B.shape[2],
                            _ptr(beta), _ptr(Cout), Cout.shape[2], Cout.shape[1] * Cout.shape[2],
                            r0, r1, c0, c1, nthreads)
    assert rc == 0, rc
    return Cout


def gemm_split(P, s, ta, tb, m, n, k, alpha, A, B, beta, C, rows=None, cols=None, nthreads=0,
               debug=False):
    """Split (sliced-integer) form; returns C, or (C, E, F, S) with debug=True
    (S: (s, n, m) int64 diagonal sums, column-major per diagonal)."""
    A = _f64(A)
    B = _f64(B)
    Cout = _f64(C).copy()
    _check_gemm(P, ta, tb, m, n, k, A, B, Cout)
    alpha = _f64(alpha)
    beta = _f64(beta)
    r0, r1 = rows if rows is not None else (0, -1)
    c0, c1 = cols if cols is not None else (0, -1)
    E = np.zeros(max(m, 1), dtype=np.int32)
    F = np.zeros(max(n, 1), dtype=np.int32)
    S = np.zeros((s, n, m), dtype=np.int64) if debug else None
    rc = lib().ref_gemm_split(P, s, ta.encode(), tb.encode(), m, n, k, _ptr(alpha), _ptr(A),
                              A.shape[2], A.shape[1] * A.shape[2], _ptr(B), B.shape[2],
                              B.shape[1] * B.shape[2], _ptr(beta), _ptr(Cout), Cout.shape[2],
                              Cout.shape[1] * Cout.shape[2], r0, r1, c0, c1, nthreads,
                              _ptr(E) if debug else None, _ptr(F) if debug else None,
                              _ptr(S) if debug else None)
    assert rc == 0, rc
    if debug:
        return Cout, E[:m], F[:n], S
    return Cout


def split_exponents(P, t, is_b, count, k, X):
    X = _f64(X)
    E = np.zeros(max(count, 1), dtype=np.int32)
    lib().ref_split_exponents(P, t.encode(), int(is_b), count, k, _ptr(X), X.shape[2],
                              X.shape[1] * X.shape[2], _ptr(E))
    return E[:count]


def split_slices(P, s, t, is_b, count, k, X, E):
    """Digits (s, count, k) int8 of op(A) rows (is_b=0) / op(B) columns."""
    X = _f64(X)
    E = np.ascontiguousarray(E, dtype=np.int32)
    D = np.zeros((s, count, k), dtype=np.int8)
    lib().ref_split_slices(P, s, t.encode(), int(is_b), count, k, _ptr(X), X.shape[2],
                           X.shape[1] * X.shape[2], _ptr(E), _ptr(D))
    return D


def split_recombine(P, s, S, ef):
    """Exact recombination of rows of anti-diagonal sums S (count, s) int64
    with scale exponents ef (count,) = E_i + F_j: (count, P) components."""
    S = np.ascontiguousarray(S, dtype=np.int64)
    ef = np.ascontiguousarray(ef, dtype=np.int32)
    count = S.shape[0]
    assert S.shape == (count, s) and ef.shape == (count,)
    out = np.zeros((max(count, 1), P))
    rc = lib().ref_split_recombine(P, s, count, _ptr(S), _ptr(ef), _ptr(out))
    if rc:
        raise ValueError(f"ref_split_recombine: {rc}")
    return out[:count]


def num_threads() -> int:
    return int(lib().ref_num_threads())
