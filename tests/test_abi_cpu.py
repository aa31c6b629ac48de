"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/mpgemm.h declares, and rejects invalid arguments on the host
(in argument order, before any GPU work)."""
import ctypes as C
import os
import re

import pytest

import paper_2101_06584_amd as mp
from paper_2101_06584_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "mpgemm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b((?:mpgemm|mp)_\w+)\s*\(", txt))
    return names


def test_library_loads_and_exports_header_symbols():
    L = mp.load()
    names = header_symbols()
    assert len(names) >= 25
    for name in names:
        assert hasattr(L, name), name
    assert set(_lib.EXPORTS) == names


def test_strerror_and_version():
    L = mp.load()
    assert L.mpgemm_version().startswith(b"mpgemm")
    for code in (0, -3, 1, 2, 3, 4, 5, 6, 99):
        assert L.mpgemm_strerror(code)


D2 = C.c_double * 2
ONE = D2(1.0, 0.0)
ZERO = D2(0.0, 0.0)
FAKE_A = C.c_void_p(0x10000000)
FAKE_B = C.c_void_p(0x20000000)
FAKE_C = C.c_void_p(0x30000000)


def call(**kw):
    a = dict(ta=b"N", tb=b"N", m=4, n=5, k=6, alpha=ONE, A=FAKE_A, lda=4, sa=24, B=FAKE_B, ldb=6,
             sb=30, beta=ZERO, C=FAKE_C, ldc=4, sc=20)
    a.update(kw)
    return mp.load().mpgemm_dd(a["ta"], a["tb"], a["m"], a["n"], a["k"], a["alpha"], a["A"], a["lda"],
                               a["sa"], a["B"], a["ldb"], a["sb"], a["beta"], a["C"], a["ldc"], a["sc"],
                               None)


@pytest.mark.parametrize("kw,code", [
    (dict(ta=b"X"), -1), (dict(tb=b"Q"), -2), (dict(m=-1), -3), (dict(n=-1), -4), (dict(k=-1), -5),
    (dict(alpha=None), -6), (dict(A=None), -7), (dict(lda=3), -8), (dict(sa=23), -9),
    (dict(B=None), -10), (dict(ldb=5), -11), (dict(sb=29), -12), (dict(beta=None), -13),
    (dict(C=None), -14), (dict(ldc=3), -15), (dict(sc=19), -16),
    (dict(ta=b"T", lda=4), -8),          # op(A) = A^T: A is k x m, needs lda >= 6
    (dict(tb=b"t", ldb=4), -11),         # op(B) = B^T: B is n x k, needs ldb >= 5
    (dict(ta=b"X", m=-1), -1),           # first invalid argument wins
])
def test_invalid_arguments(kw, code):
    assert call(**kw) == code


def test_quick_returns_need_no_gpu():
    # m == 0 / n == 0: nothing to do, pointers never touched
    assert call(m=0, A=None, C=None, ldc=1, sc=5, lda=1, sa=6) == 0
    assert call(n=0, B=None, C=None, sc=0, sb=0, ldb=6) == 0
    # alpha == 0 and beta == 1: quick return; A/B may be NULL
    assert call(alpha=ZERO, beta=ONE, A=None, B=None) == 0
    # k == 0 and beta == 1
    assert call(k=0, beta=ONE, A=None, B=None, lda=4, sa=0, ldb=1, sb=5) == 0


def test_aliasing_rejected():
    assert call(C=FAKE_A) == _lib.ERR_ALIAS


def test_ex_options_validated():
    L = mp.load()
    o = mp.make_opts("split", slices=41)
    rc = L.mpgemm_dd_ex(b"N", b"N", 4, 5, 6, ONE, FAKE_A, 4, 24, FAKE_B, 6, 30, ZERO, FAKE_C, 4, 20,
                        None, C.byref(o))
    assert rc == -18
    o = mp.make_opts("split", slices=16)          # no workspace
    rc = L.mpgemm_dd_ex(b"N", b"N", 4, 5, 6, ONE, FAKE_A, 4, 24, FAKE_B, 6, 30, ZERO, FAKE_C, 4, 20,
                        None, C.byref(o))
    assert rc == _lib.ERR_WORKSPACE
    o = mp.make_opts("split", slices=40)          # k * s beyond exact int32 accumulation
    rc = L.mpgemm_dd_ex(b"N", b"N", 4, 5, 20000, ONE, FAKE_A, 4, 80000, FAKE_B, 20000, 100000, ZERO,
                        FAKE_C, 4, 20, None, C.byref(o))
    assert rc == _lib.ERR_UNSUPPORTED


def test_crt_form_host_rules():
    """Residue form: feasibility by modulus count, workspace checks, all on
    the host before any GPU work."""
    L = mp.load()
    D4 = C.c_double * 4
    one4, zero4 = D4(1.0, 0, 0, 0), D4(0, 0, 0, 0)
    o = mp.make_opts("crt", slices=33)            # QD beyond two levels of 16 digits
    rc = L.mpgemm_qd_ex(b"N", b"N", 4, 5, 6, one4, FAKE_A, 4, 24, FAKE_B, 6, 30, zero4, FAKE_C, 4, 20,
                        None, C.byref(o))
    assert rc == _lib.ERR_UNSUPPORTED
    assert L.mpgemm_workspace_bytes(4, 5, 4, 5, 6, 33, -1) == 0
    assert L.mpgemm_workspace_bytes(4, 5, 4, 5, 6, 0, -1) > 0       # QD default s = 31: two levels
    o = mp.make_opts("crt", slices=25)            # s > 24
    rc = L.mpgemm_dd_ex(b"N", b"N", 4, 5, 6, ONE, FAKE_A, 4, 24, FAKE_B, 6, 30, ZERO, FAKE_C, 4, 20,
                        None, C.byref(o))
    assert rc == _lib.ERR_UNSUPPORTED
    o = mp.make_opts("crt")                       # k beyond exact int32 sums of byte products
    rc = L.mpgemm_dd_ex(b"N", b"N", 4, 5, 131072, ONE, FAKE_A, 4, 4 * 131072, FAKE_B, 131072,
                        5 * 131072, ZERO, FAKE_C, 4, 20, None, C.byref(o))
    assert rc == _lib.ERR_UNSUPPORTED
    o = mp.make_opts("crt")                       # feasible, but no workspace
    rc = L.mpgemm_dd_ex(b"N", b"N", 4, 5, 6, ONE, FAKE_A, 4, 24, FAKE_B, 6, 30, ZERO, FAKE_C, 4, 20,
                        None, C.byref(o))
    assert rc == _lib.ERR_WORKSPACE
    o = mp.make_opts("crt", variant=1)
    rc = L.mpgemm_td_ex(b"N", b"N", 4, 5, 6, D4(1, 0, 0, 0), FAKE_A, 4, 24, FAKE_B, 6, 30, D4(), FAKE_C,
                        4, 20, None, C.byref(o))
    assert rc == _lib.ERR_UNSUPPORTED
    # workspace: exponents, N residue planes per operand, N result bytes per entry
    b16 = L.mpgemm_workspace_bytes(2, 5, 100, 100, 4096, 16, 2)      # DD: 32 moduli, 128 x 128 tiles
    assert b16 >= 32 * (128 * 4096 * 2 + 128 * 128)
    b23 = L.mpgemm_workspace_bytes(3, 5, 100, 100, 4096, 0, 2)       # TD default s = 23: 48 moduli
    assert b23 >= 48 * (128 * 4096 * 2 + 128 * 128) > b16
    assert mp.num_configs(2, "crt") == 3
    assert (mp.crt_moduli(2, 4096), mp.crt_moduli(3, 4096), mp.crt_moduli(3, 65536)) == (32, 48, 49)
    assert mp.crt_moduli(4, 129, 20) == 40 and mp.crt_moduli(2, 131072) == 0
    # QD with more than 24 digits: two levels, three products of N moduli each
    assert (mp.crt_moduli(4, 100), mp.crt_moduli(4, 4096), mp.crt_moduli(4, 50, 25)) == (93, 96, 75)
    assert mp.crt_moduli(4, 131071, 32) == 99 and mp.crt_moduli(3, 4096, 31) == 0
    assert L.mpgemm_crt_moduli(7, 10, 0) == -1


def test_auto_form_workspace_fits_either_split_form():
    """FORM_AUTO's workspace is the larger of the two split forms' needs
    (the residue form's where it applies, the triangular form's elsewhere)."""
    for P, m, n, k, s in [(2, 256, 256, 256, 0), (3, 1000, 300, 700, 0), (4, 512, 512, 512, 0),
                          (2, 300, 300, 4096, 20), (4, 256, 256, 256, 33)]:
        split = mp.workspace_bytes(P, "split", m, n, k, s)
        crt = mp.workspace_bytes(P, "crt", m, n, k, s)
        assert mp.workspace_bytes(P, "auto", m, n, k, s) == max(split, crt), (P, m, n, k, s)
    assert mp.workspace_bytes(4, "crt", 256, 256, 256, 33) == 0          # no residue form: split's
    assert mp.workspace_bytes(4, "auto", 256, 256, 256, 33) == mp.workspace_bytes(4, "split", 256, 256, 256, 33)


def test_vec_validation():
    L = mp.load()
    assert L.mp_vec_td_add(-1, None, 0, None, 0, None, 0, None) == -1
    assert L.mp_vec_td_add(10, None, 10, FAKE_B, 10, FAKE_C, 10, None) == -2
    assert L.mp_vec_qd_mul(10, FAKE_A, 9, FAKE_B, 10, FAKE_C, 10, None) == -3
    assert L.mp_vec_dd_mul(0, None, 0, None, 0, None, 0, None) == 0


def test_workspace_bytes_and_layout():
    L = mp.load()
    assert L.mpgemm_workspace_bytes(2, 0, 100, 100, 100, 0, -1) == 0
    b = L.mpgemm_workspace_bytes(2, 1, 100, 100, 100, 16, -1)
    lay = mp.split_layout(2, 100, 100, 100, 16)
    assert lay["Mp"] % 64 == 0 and lay["Np"] % 64 == 0 and lay["Kp"] % 64 == 0
    assert lay["S"] + 4 * 16 * lay["Mp"] * lay["Np"] <= b
    assert lay["DA"] >= lay["F"] + 4 * lay["Np"]
    assert L.mpgemm_workspace_bytes(5, 1, 1, 1, 1, 0, -1) == 0
    assert mp.num_configs(2, "plain") >= 2 and mp.num_configs(4, "split") >= 1


def test_batch_plan_validation():
    L = mp.load()
    h = C.c_void_p()
    assert L.mpgemm_batch_plan_create(7, 0, None, None, None, C.byref(h)) == -1
    assert L.mpgemm_batch_plan_create(2, -1, None, None, None, C.byref(h)) == -2
    assert L.mpgemm_batch_plan_create(2, 3, None, None, None, C.byref(h)) == -3
    arr = (_lib.Problem * 2)()
    for x in arr:
        x.transa = b"N"; x.transb = b"N"; x.m = 4; x.n = 4; x.k = 4
        x.alpha[0] = 1.0
        x.A, x.lda, x.a_plane_stride = FAKE_A, 4, 16
        x.B, x.ldb, x.b_plane_stride = FAKE_B, 4, 16
        x.C, x.ldc, x.c_plane_stride = FAKE_C, 4, 16
    # forms: plain, auto and residue only; options in range; the residue form
    # needs a residue product for every problem that multiplies (none for k
    # beyond 131071, nor for s > 24 below QD, which alone has two levels)
    def opts(form, slices=0):
        o = _lib.Opts()
        o.form, o.slices, o.tile = form, slices, -1
        return o
    for form in (_lib.FORM_SPLIT_I8, _lib.FORM_STRASSEN):
        assert L.mpgemm_batch_plan_create(2, 2, arr, C.byref(opts(form, 16)), None, C.byref(h)) == \
            _lib.ERR_UNSUPPORTED
    assert L.mpgemm_batch_plan_create(2, 2, arr, C.byref(opts(_lib.FORM_SPLIT_CRT, 99)), None, C.byref(h)) == -4
    for P in (2, 3):
        assert L.mpgemm_batch_plan_create(P, 2, arr, C.byref(opts(_lib.FORM_SPLIT_CRT, 25)), None,
                                          C.byref(h)) == _lib.ERR_UNSUPPORTED
    assert L.mpgemm_crt_moduli(4, 4, 25) > 0 and L.mpgemm_crt_moduli(4, 4, 31) > 0
    big = (_lib.Problem * 1)()
    x = big[0]
    x.transa = b"N"; x.transb = b"N"; x.m = 4; x.n = 4; x.k = 131072
    x.alpha[0] = 1.0
    x.A, x.lda, x.a_plane_stride = FAKE_A, 4, 4 * 131072
    x.B, x.ldb, x.b_plane_stride = FAKE_B, 131072, 4 * 131072
    x.C, x.ldc, x.c_plane_stride = FAKE_C, 4, 16
    for P, sl in ((2, 16), (4, 0), (4, 20)):
        assert L.mpgemm_batch_plan_create(P, 1, big, C.byref(opts(_lib.FORM_SPLIT_CRT, sl)), None,
                                          C.byref(h)) == _lib.ERR_UNSUPPORTED
    arr[1].ldc = 2
    assert L.mpgemm_batch_plan_create(2, 2, arr, None, None, C.byref(h)) == -1001


def test_tune_slices_validation():
    L = mp.load()
    s, r = C.c_int(), C.c_double()
    assert L.mpgemm_tune_slices(2, b"N", b"N", 4, 4, 4, FAKE_A, 4, 16, FAKE_B, 4, 16, 0.0, 10, 20,
                                None, C.byref(s), C.byref(r)) == -13
    assert L.mpgemm_tune_slices(2, b"N", b"N", 4, 4, 4, FAKE_A, 4, 16, FAKE_B, 4, 16, 1.0, 10, 5,
                                None, C.byref(s), C.byref(r)) == -15


def test_blas_rejects_invalid_arguments_on_the_host():
    """axpy, dot and gemv validate in argument order before any GPU work."""
    L = mp.load()
    d2 = (C.c_double * 2)(1.0, 0.0)
    fake = C.c_void_p(4096)
    assert L.mp_axpy_dd(-1, d2, fake, 0, fake, 0, None) == -1
    assert L.mp_axpy_dd(4, None, fake, 4, fake, 4, None) == -2
    assert L.mp_axpy_dd(4, d2, fake, 3, fake, 4, None) == -4
    assert L.mp_axpy_dd(4, d2, fake, 4, fake, 3, None) == -6
    assert L.mp_dot_workspace_bytes(2, 64) == 0
    assert L.mp_dot_workspace_bytes(2, 65) == 2 * 2 * 8
    assert L.mp_dot_workspace_bytes(4, 64 * 64 * 64 + 1) == 8 * 4 * (4097 + 65 + 2)
    assert L.mp_dot_dd(5, fake, 4, fake, 5, fake, None, 0, None) == -3
    assert L.mp_dot_dd(5, fake, 5, fake, 5, None, None, 0, None) == -6
    assert L.mp_dot_dd(65, fake, 65, fake, 65, fake, None, 0, None) == -7
    assert L.mp_dot_dd(65, fake, 65, fake, 65, fake, fake, 8, None) == _lib.ERR_WORKSPACE
    assert L.mp_gemv_dd(b"X", 4, 4, d2, fake, 4, 16, fake, 4, d2, fake, 4, None) == -1
    assert L.mp_gemv_dd(b"N", 4, 4, d2, fake, 3, 16, fake, 4, d2, fake, 4, None) == -6
    assert L.mp_gemv_dd(b"N", 4, 4, d2, fake, 4, 15, fake, 4, d2, fake, 4, None) == -7
    assert L.mp_gemv_dd(b"T", 4, 6, d2, fake, 4, 24, fake, 3, d2, fake, 6, None) == -9
    assert L.mp_gemv_dd(b"N", 4, 6, d2, fake, 4, 24, fake, 6, d2, fake, 3, None) == -12
    # y overlapping A
    assert L.mp_gemv_dd(b"N", 4, 4, d2, fake, 4, 16, C.c_void_p(9 * 4096), 4, d2,
                        C.c_void_p(4096 + 8), 4, None) == _lib.ERR_ALIAS


def test_grouped_validation():
    """The grouped calls check their arguments (and every problem) on the
    host before any GPU work."""
    L = mp.load()
    assert L.mpgemm_dd_grouped(-1, None, None, None) == -1
    assert L.mpgemm_td_grouped(2, None, None, None) == -2
    assert L.mpgemm_qd_grouped(0, None, None, None) == 0          # nothing to do
    arr = (_lib.Problem * 2)()
    for x in arr:
        x.transa = b"N"; x.transb = b"N"; x.m = 4; x.n = 4; x.k = 4
        x.alpha[0] = 1.0
        x.A, x.lda, x.a_plane_stride = FAKE_A, 4, 16
        x.B, x.ldb, x.b_plane_stride = FAKE_B, 4, 16
        x.C, x.ldc, x.c_plane_stride = FAKE_C, 4, 16
    split = _lib.Opts()
    split.form = _lib.FORM_SPLIT_I8
    assert L.mpgemm_dd_grouped(2, arr, C.byref(split), None) == -3     # plain, auto, residue only
    variant = _lib.Opts()
    variant.variant = 1
    assert L.mpgemm_td_grouped(2, arr, C.byref(variant), None) == -3
    arr[1].ldb = 1
    assert L.mpgemm_dd_grouped(2, arr, None, None) == -1001


CHILD = r'''
import ctypes as C, sys
L = C.CDLL(sys.argv[1])
L.mpgemm_workspace_bytes.restype = C.c_size_t
L.mpgemm_workspace_bytes.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int]
n = 300
print(L.mpgemm_workspace_bytes(2, 1, n, n, n, 16, -1), L.mpgemm_workspace_bytes(2, 1, n, n, n, 16, 0),
      L.mpgemm_workspace_bytes(2, 1, n, n, n, 16, 1))
'''


def _child(env_extra):
    """Workspace bytes of the DD split form at n = 300 (tuned tile, tile 0,
    tile 1) as a C-only caller sees them: ctypes on the shared library in a
    fresh process, no Python binding, no torch."""
    import subprocess
    import sys
    env = {k: v for k, v in os.environ.items() if not k.startswith("MPGEMM_")}
    env.update(env_extra)
    out = subprocess.run([sys.executable, "-c", CHILD, _lib.LIB_PATH], env=env, capture_output=True,
                         text=True, check=True).stdout.split()
    return [int(v) for v in out]


def test_c_callers_get_the_tuned_tiles(tmp_path):
    """The library loads the tuning table by itself: an entry for the DD
    split form at 256^3 (the log2 bucket of n = 300) selects that tile for a
    C-only caller; entries with another configuration signature or a file
    of another format are ignored; MPGEMM_NO_TUNED_TABLE turns it off."""
    L = mp.load()
    sig = None
    with open(_lib.TUNED_TABLE) as f:
        header = f.readline()
        for line in f:
            v = line.split()
            if v[1] == "1":
                sig = v[6]
    assert header.startswith("# mpgemm tuning table v2 arch=gfx950")
    assert sig is not None
    _, t0, t1 = _child({"MPGEMM_NO_TUNED_TABLE": "1"})
    assert t0 != t1
    for tile, want in ((0, t0), (1, t1)):
        p = tmp_path / f"table{tile}.txt"
        p.write_text(header + f"2 1 8 8 8 {tile} {sig}\n")
        assert _child({"MPGEMM_AUTOTUNE_CACHE": str(p)})[0] == want
    default = _child({"MPGEMM_NO_TUNED_TABLE": "1"})[0]
    bad_sig = tmp_path / "bad_sig.txt"
    bad_sig.write_text(header + "2 1 8 8 8 0 00000000\n2 1 8 8 8 1 00000000\n")
    assert _child({"MPGEMM_AUTOTUNE_CACHE": str(bad_sig)})[0] == default
    old = tmp_path / "old.txt"
    old.write_text("# mpgemm tuning table v1 gfx950: prec form log2m log2n log2k tile\n2 1 8 8 8 0\n")
    assert _child({"MPGEMM_AUTOTUNE_CACHE": str(old)})[0] == default
    assert L.mpgemm_autotune_load(str(old).encode()) == _lib.ERR_UNSUPPORTED
    # save writes the header and a signature per entry
    out = tmp_path / "saved.txt"
    assert L.mpgemm_autotune_save(str(out).encode()) == 0
    lines = out.read_text().splitlines()
    assert lines[0].startswith("# mpgemm tuning table v2 arch=gfx950")
    assert all(len(l.split()) == 7 for l in lines[1:])


def test_row_major_matmul_argument_checks():
    """Shape checks of the row-major entry happen before any device call."""
    import torch
    import paper_2101_06584_amd as mp
    A = torch.zeros((2, 4, 5), dtype=torch.float64)
    B = torch.zeros((2, 6, 3), dtype=torch.float64)
    with pytest.raises(ValueError, match="inner dimensions"):
        mp.matmul(2, A, B)
    with pytest.raises(ValueError, match="expected A"):
        mp.matmul(3, A, torch.zeros((2, 5, 3), dtype=torch.float64))
    with pytest.raises(ValueError, match="beta != 0"):
        mp.matmul(2, A, torch.zeros((2, 5, 3), dtype=torch.float64), beta=(0.5, 0.0))
    with pytest.raises(ValueError, match="expected C_"):
        mp.matmul(2, A, torch.zeros((2, 5, 3), dtype=torch.float64), torch.zeros((2, 3, 4), dtype=torch.float64))
