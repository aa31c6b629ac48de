"""mpgemm_ex_noalloc (the _ex call with the library's static scratch buffer)
against the _ex entry point with a workspace of its own: bit for bit, for
every form that uses scratch, two calls in a row on one stream with the
second smaller (the buffer keeps the first call's contents), plus the
host-side rejections (scratch too small, a workspace passed, argument
numbering)."""
import numpy as np
import pytest

from paper_2101_06584_amd import _lib
from tests import synth
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu

FAM = 9


def make(P, ta, tb, m, n, k):
    A = synth.mp_matrix(FAM, "A", P, *((m, k) if ta == "N" else (k, m)))
    B = synth.mp_matrix(FAM, "B", P, *((k, n) if tb == "N" else (n, k)))
    C = synth.mp_matrix(FAM, "C", P, m, n)
    return A, B, C, synth.mp_scalar(FAM, "alpha", P), synth.mp_scalar(FAM, "beta", P)


def both(gpu_lib, P, form, ta, tb, m, n, k, slices=0, levels=0):
    """(no-alloc result, _ex result with its own workspace) on the same inputs."""
    A, B, C, alpha, beta = make(P, ta, tb, m, n, k)
    wsf = {"crt": "crt", "split": "split", "auto": "auto", "strassen": "strassen"}[form]
    need = gpu_lib.workspace_bytes(P, form, m, n, k, levels if form == "strassen" else slices)
    if form != "auto":
        assert 0 < need <= _lib.STATIC_SCRATCH_BYTES, (form, need)
    dA, dB = dev(A), dev(B)
    c1 = dev(C)
    note("noalloc", P, form, ta, tb, (m, n, k), "scratch need", need)
    gpu_lib.gemm_noalloc(P, ta, tb, m, n, k, alpha, dA, dB, beta, c1, form=form, slices=slices,
                         levels=levels)
    got = host(c1)
    ws = gpu_lib.alloc_workspace(P, m, n, k, slices, device="cuda", form=wsf, levels=levels)
    c2 = dev(C)
    gpu_lib.gemm(P, ta, tb, m, n, k, alpha, dA, dB, beta, c2, form=form, slices=slices, workspace=ws,
                 levels=levels)
    want = host(c2)
    return got, want, C


# (first call, second call): the second smaller, other transposes
CASES = {
    "crt": [((2, "N", "N", 600, 520, 560), (2, "T", "N", 70, 45, 33)),
            ((3, "N", "T", 400, 380, 410), (3, "T", "T", 65, 129, 31)),
            ((4, "T", "N", 330, 300, 350), (4, "N", "N", 40, 41, 129))],
    "split": [((2, "N", "N", 520, 500, 530), (2, "N", "T", 90, 70, 60)),
              ((3, "T", "N", 400, 390, 380), (3, "N", "N", 33, 65, 100)),
              ((4, "N", "T", 330, 320, 300), (4, "T", "T", 17, 19, 70))],
    "strassen": [((2, "N", "N", 256, 320, 192), (2, "T", "N", 64, 32, 96)),
                 ((4, "N", "T", 192, 128, 256), (4, "N", "N", 32, 64, 32))],
    "auto": [((2, "N", "N", 500, 480, 470), (2, "T", "T", 130, 129, 128)),
             ((3, "N", "N", 2000, 96, 100), (3, "N", "N", 300, 97, 96))],
}


@pytest.mark.parametrize("form", ["crt", "split", "strassen", "auto"])
def test_two_calls_match_the_workspace_entry_point(gpu_lib, form):
    for first, second in CASES[form]:
        for P, ta, tb, m, n, k in (first, second):
            levels = 2 if form == "strassen" else 0
            # the auto form takes a split form only with the digit count given
            slices = gpu_lib.DEFAULT_SLICES[P] if form == "auto" else 0
            got, want, C = both(gpu_lib, P, form, ta, tb, m, n, k, slices=slices, levels=levels)
            assert np.array_equal(got, want), (form, P, (m, n, k))
            assert not np.array_equal(got, C)      # the call wrote C


def test_plain_form_and_td_variant(gpu_lib):
    for P, ta, tb, m, n, k, variant in ((2, "N", "T", 77, 66, 55, 0), (3, "T", "N", 50, 40, 30, 3)):
        A, B, C, alpha, beta = make(P, ta, tb, m, n, k)
        dA, dB, c1, c2 = dev(A), dev(B), dev(C), dev(C)
        note("noalloc plain", P, (m, n, k), "variant", variant)
        gpu_lib.gemm_noalloc(P, ta, tb, m, n, k, alpha, dA, dB, beta, c1, form="plain", variant=variant)
        gpu_lib.gemm(P, ta, tb, m, n, k, alpha, dA, dB, beta, c2, form="plain", variant=variant)
        assert np.array_equal(host(c1), host(c2))


def test_host_side_rejections(gpu_lib):
    P, m, n, k = 2, 1024, 1024, 1024
    need = gpu_lib.workspace_bytes(P, "crt", m, n, k)
    assert need > _lib.STATIC_SCRATCH_BYTES
    A, B, C, alpha, beta = make(P, "N", "N", 8, 8, 8)
    small = dev(C)
    # sizes beyond the buffer: rejected before any GPU work (tensors are
    # never touched, so small stand-ins of the right type suffice)
    big = dev(np.zeros((P, n, m)))
    bigA = dev(np.zeros((P, k, m)))
    bigB = dev(np.zeros((P, n, k)))
    note("noalloc too big", P, (m, n, k), need)
    for form in ("crt", "split"):
        rc = gpu_lib.gemm_noalloc_raw(P, "N", "N", m, n, k, alpha, bigA, bigB, beta, big, form=form)
        assert rc == _lib.ERR_SCRATCH, (form, rc)
    # form auto never rejects: it falls back to a form that fits (checked
    # against the workspace entry point's plain result)
    gpu_lib.gemm_noalloc(P, "N", "N", 8, 8, 8, alpha, dev(A), dev(B), beta, small, form="auto")
    want = dev(C)
    gpu_lib.gemm(P, "N", "N", 8, 8, 8, alpha, dev(A), dev(B), beta, want, form="plain")
    assert np.array_equal(host(small), host(want))
    # invalid arguments: prec is argument 1, the rest shift by one
    L = gpu_lib.load()
    import ctypes as C_

    one = (C_.c_double * 4)(1.0, 0, 0, 0)
    o = _lib.Opts()
    o.form = _lib.FORM_SPLIT_CRT
    s0 = C_.c_void_p(0)
    a = C_.c_void_p(bigA.data_ptr())
    b = C_.c_void_p(bigB.data_ptr())
    c = C_.c_void_p(big.data_ptr())
    assert L.mpgemm_ex_noalloc(5, b"N", b"N", 8, 8, 8, one, a, 8, 64, b, 8, 64, one, c, 8, 64, s0,
                               C_.byref(o)) == -1
    assert L.mpgemm_ex_noalloc(2, b"X", b"N", 8, 8, 8, one, a, 8, 64, b, 8, 64, one, c, 8, 64, s0,
                               C_.byref(o)) == -2
    assert L.mpgemm_ex_noalloc(2, b"N", b"N", 8, 8, 8, one, a, 4, 64, b, 8, 64, one, c, 8, 64, s0,
                               C_.byref(o)) == -9
    assert L.mpgemm_ex_noalloc(2, b"N", b"N", 8, 8, 8, one, a, 8, 64, b, 8, 64, one, c, 8, 64, s0,
                               None) == -19
    o.workspace = a
    o.workspace_bytes = 256
    assert L.mpgemm_ex_noalloc(2, b"N", b"N", 8, 8, 8, one, a, 8, 64, b, 8, 64, one, c, 8, 64, s0,
                               C_.byref(o)) == -19
