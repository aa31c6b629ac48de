"""ctypes declarations of libmpgemm's C ABI (include/mpgemm.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Loading fails loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpgemm.so")
# tile choices measured on MI355X by paper_2101_06584_amd/tune.py; the library
# loads this file (or the one MPGEMM_AUTOTUNE_CACHE names) by itself
TUNED_TABLE = os.path.join(_HERE, "tuned_gfx950.txt")

_i64, _int, _ch, _vp, _sz, _dbl = C.c_int64, C.c_int, C.c_char, C.c_void_p, C.c_size_t, C.c_double
_P = C.POINTER

ERR_HIP, ERR_WORKSPACE, ERR_UNSUPPORTED, ERR_GRAPH, ERR_ALIAS, ERR_NOMEM, ERR_SCRATCH = 1, 2, 3, 4, 5, 6, 7
STATIC_SCRATCH_BYTES = 64 << 20   # MPGEMM_STATIC_SCRATCH_BYTES
FORM_PLAIN, FORM_SPLIT_I8, FORM_AUTO, FORM_STRASSEN, FORM_SPLIT_CRT = 0, 1, 2, 4, 5
TD_ADD_ACCURATE, TD_MULQ = 1, 2


class Opts(C.Structure):
    _fields_ = [("form", _int), ("slices", _int), ("tile", _int), ("variant", _int),
                ("workspace", _vp), ("workspace_bytes", _sz), ("levels", _int)]


class Problem(C.Structure):
    _fields_ = [("transa", _ch), ("transb", _ch), ("m", _i64), ("n", _i64), ("k", _i64),
                ("alpha", _dbl * 4), ("beta", _dbl * 4),
                ("A", _vp), ("lda", _i64), ("a_plane_stride", _i64),
                ("B", _vp), ("ldb", _i64), ("b_plane_stride", _i64),
                ("C", _vp), ("ldc", _i64), ("c_plane_stride", _i64)]


_GEMM_ARGS = [_ch, _ch, _i64, _i64, _i64, _P(_dbl), _vp, _i64, _i64, _vp, _i64, _i64, _P(_dbl),
              _vp, _i64, _i64, _vp]
_VEC_ARGS = [_i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp]

EXPORTS = {
    "mpgemm_dd": (_GEMM_ARGS, _int), "mpgemm_td": (_GEMM_ARGS, _int), "mpgemm_qd": (_GEMM_ARGS, _int),
    "mpgemm_dd_ex": (_GEMM_ARGS + [_P(Opts)], _int),
    "mpgemm_td_ex": (_GEMM_ARGS + [_P(Opts)], _int),
    "mpgemm_qd_ex": (_GEMM_ARGS + [_P(Opts)], _int),
    "mpgemm_ex_noalloc": ([_int] + _GEMM_ARGS + [_P(Opts)], _int),
    "mpgemm_workspace_bytes": ([_int, _int, _i64, _i64, _i64, _int, _int], _sz),
    "mpgemm_crt_moduli": ([_int, _i64, _int], _int),
    "mp_vec_dd_add": (_VEC_ARGS, _int), "mp_vec_dd_mul": (_VEC_ARGS, _int),
    "mp_vec_td_add": (_VEC_ARGS, _int), "mp_vec_td_mul": (_VEC_ARGS, _int),
    "mp_vec_qd_add": (_VEC_ARGS, _int), "mp_vec_qd_mul": (_VEC_ARGS, _int),
    "mp_vec_td_add_acc": (_VEC_ARGS, _int), "mp_vec_td_mulq": (_VEC_ARGS, _int),
    "mp_axpy_dd": ([_i64, _P(_dbl), _vp, _i64, _vp, _i64, _vp], _int),
    "mp_axpy_td": ([_i64, _P(_dbl), _vp, _i64, _vp, _i64, _vp], _int),
    "mp_axpy_qd": ([_i64, _P(_dbl), _vp, _i64, _vp, _i64, _vp], _int),
    "mp_dot_workspace_bytes": ([_int, _i64], _sz),
    "mp_dot_dd": ([_i64, _vp, _i64, _vp, _i64, _vp, _vp, _sz, _vp], _int),
    "mp_dot_td": ([_i64, _vp, _i64, _vp, _i64, _vp, _vp, _sz, _vp], _int),
    "mp_dot_qd": ([_i64, _vp, _i64, _vp, _i64, _vp, _vp, _sz, _vp], _int),
    "mp_gemv_dd": ([_ch, _i64, _i64, _P(_dbl), _vp, _i64, _i64, _vp, _i64, _P(_dbl), _vp, _i64, _vp], _int),
    "mp_gemv_td": ([_ch, _i64, _i64, _P(_dbl), _vp, _i64, _i64, _vp, _i64, _P(_dbl), _vp, _i64, _vp], _int),
    "mp_gemv_qd": ([_ch, _i64, _i64, _P(_dbl), _vp, _i64, _i64, _vp, _i64, _P(_dbl), _vp, _i64, _vp], _int),
    "mpgemm_batch_plan_create": ([_int, _i64, _P(Problem), _P(Opts), _vp, _P(_vp)], _int),
    "mpgemm_batch_plan_run": ([_vp, _vp], _int),
    "mpgemm_batch_plan_launch": ([_vp, _vp], _int),
    "mpgemm_batch_plan_info": ([_vp, _P(_i64), _P(_int), _P(_int)], _int),
    "mpgemm_batch_plan_residue_info": ([_vp, _P(_i64), _P(_int), _P(_int), _P(_sz)], _int),
    "mpgemm_batch_plan_destroy": ([_vp], _int),
    "mpgemm_dd_grouped": ([_i64, _P(Problem), _P(Opts), _vp], _int),
    "mpgemm_td_grouped": ([_i64, _P(Problem), _P(Opts), _vp], _int),
    "mpgemm_qd_grouped": ([_i64, _P(Problem), _P(Opts), _vp], _int),
    "mpgemm_autotune": ([_int, _int, _i64, _i64, _i64, _int, _vp, _P(_int)], _int),
    "mpgemm_batch_autotune": ([_int, _i64, _P(Problem), _vp, _P(_int)], _int),
    "mpgemm_autotune_set": ([_int, _int, _i64, _i64, _i64, _int], _int),
    "mpgemm_autotune_save": ([C.c_char_p], _int),
    "mpgemm_autotune_load": ([C.c_char_p], _int),
    "mpgemm_num_configs": ([_int, _int], _int),
    "mpgemm_tune_slices": ([_int, _ch, _ch, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _i64,
                            _dbl, _int, _int, _vp, _P(_int), _P(_dbl)], _int),
    "mpgemm_split_layout": ([_int, _i64, _i64, _i64, _int, _int, _P(_sz), _P(_sz), _P(_sz),
                             _P(_sz), _P(_sz), _P(_i64), _P(_i64), _P(_i64)], _int),
    "mpgemm_split_stages": ([_int, _int] + _GEMM_ARGS + [_P(Opts)], _int),
    "mpgemm_probe_peak": ([_int, _vp, _P(_dbl)], _int),
    "mpgemm_strerror": ([_int], C.c_char_p),
    "mpgemm_version": ([], C.c_char_p),
    "mpgemm_finalize": ([], None),
}

_LIB = None


def load(path: str | None = None):
    """Load libmpgemm.so and declare every exported symbol; raises if missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libmpgemm.so not built ({p}); run __graft_entry__.build() "
                           "or python paper_2101_06584_amd/build.py")
    lib = C.CDLL(p)
    for name, (args, res) in EXPORTS.items():
        fn = getattr(lib, name)          # AttributeError if a symbol is missing
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def strerror(code: int) -> str:
    return load().mpgemm_strerror(code).decode()
