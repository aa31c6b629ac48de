"""Python binding of libmpgemm with PyTorch used only for device memory and
streams.  Matrices are float64 CUDA tensors of shape (P, cols, ld): P
column-major component planes (element (i, j) of component p is t[p, j, i]),
i.e. the library's storage with plane stride cols * ld.  Every call only
marshals arguments; the work runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import torch

from . import _lib

PREC = {"dd": 2, "td": 3, "qd": 4, 2: 2, 3: 3, 4: 4}
FORMS = {"plain": _lib.FORM_PLAIN, "split": _lib.FORM_SPLIT_I8, "auto": _lib.FORM_AUTO,
         "strassen": _lib.FORM_STRASSEN, "crt": _lib.FORM_SPLIT_CRT}
DEFAULT_SLICES = {2: 16, 3: 23, 4: 31}
_NAME = {2: "dd", 3: "td", 4: "qd"}


class MPGemmError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: error {code}: {_lib.strerror(code)}")


def load():
    return _lib.load()


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise MPGemmError(rc, what)


def _stream(stream) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _mat(t: torch.Tensor | None, P: int):
    """(pointer, ld, plane stride) of a (P, cols, ld) component-plane tensor."""
    if t is None:
        return None, 1, 1
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("matrices must be float64 CUDA tensors")
    if t.dim() != 3 or t.shape[0] != P:
        raise ValueError(f"expected shape (P={P}, cols, ld), got {tuple(t.shape)}")
    if t.stride(2) != 1 or t.stride(1) < t.shape[2] and t.shape[1] > 1:
        raise ValueError("component planes must be column-major with unit stride along rows")
    ld = max(t.stride(1), 1) if t.shape[1] > 1 else max(t.shape[2], 1)
    ps = t.stride(0) if P > 1 else ld * t.shape[1]
    return C.c_void_p(t.data_ptr()), ld, ps


def _scalar(v: Sequence[float], P: int):
    vals = [float(x) for x in v] + [0.0] * (P - len(v))
    return (C.c_double * P)(*vals[:P])


TD_VARIANTS = {"default": 0, "add_acc": _lib.TD_ADD_ACCURATE, "mulq": _lib.TD_MULQ,
               "add_acc+mulq": _lib.TD_ADD_ACCURATE | _lib.TD_MULQ}


def make_opts(form="plain", slices=0, tile=-1, workspace: torch.Tensor | None = None, variant=0,
              levels=0):
    o = _lib.Opts()
    o.levels = int(levels)
    o.form = FORMS[form] if isinstance(form, str) else int(form)
    o.slices = int(slices)
    o.tile = int(tile)
    o.variant = TD_VARIANTS[variant] if isinstance(variant, str) else int(variant)
    if workspace is not None:
        o.workspace = C.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    else:
        o.workspace = None
        o.workspace_bytes = 0
    return o


def crt_moduli(prec, k, slices=0) -> int:
    """Moduli (INT8 products) of the residue form for inner dimension k and
    `slices` digits (0 = default); 0 when it does not apply."""
    return int(_lib.load().mpgemm_crt_moduli(PREC[prec], k, slices))


def workspace_bytes(prec, form, m, n, k, slices=0, tile=-1) -> int:
    P = PREC[prec]
    f = FORMS[form] if isinstance(form, str) else int(form)
    return int(_lib.load().mpgemm_workspace_bytes(P, f, m, n, k, slices, tile))


def alloc_workspace(prec, m, n, k, slices=0, tile=-1, device=None, form="split", levels=0) -> torch.Tensor:
    """Device workspace for the split form (slices, tile), with form="crt"
    for its residue form, form="auto" for either, or with form="strassen" for
    `levels` levels of Strassen's method."""
    if form == "strassen":
        nbytes = workspace_bytes(prec, "strassen", m, n, k, levels, -1)
    elif form in ("crt", "auto"):
        nbytes = workspace_bytes(prec, form, m, n, k, slices, tile)
    else:
        nbytes = workspace_bytes(prec, "split", m, n, k, slices, tile)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device or "cuda")


def gemm_raw(prec, transa, transb, m, n, k, alpha, A, B, beta, C_, *, form=None, slices=0,
             tile=-1, workspace=None, stream=None, variant=0, levels=0) -> int:
    """Calls mpgemm_{dd,td,qd}[_ex]; returns the library's status code.
    variant (TD, plain form): "add_acc" (Algorithm 3), "mulq" (TDmulq), both,
    or the MPGEMM_TD_* bits."""
    P = PREC[prec]
    L = _lib.load()
    a, lda, sa = _mat(A, P)
    b, ldb, sb = _mat(B, P)
    c, ldc, sc = _mat(C_, P)
    args = [transa.encode(), transb.encode(), m, n, k, _scalar(alpha, P), a, lda, sa, b, ldb, sb,
            _scalar(beta, P), c, ldc, sc, _stream(stream)]
    name = "mpgemm_" + _NAME[P]
    if form is None and not variant and tile == -1 and workspace is None and not levels:
        return getattr(L, name)(*args)
    # any option given (a tile, a workspace, ...) goes through the _ex call,
    # so that it is never dropped silently
    return getattr(L, name + "_ex")(*args, C.byref(make_opts(form or "plain", slices, tile, workspace,
                                                               variant, levels)))


def gemm_noalloc_raw(prec, transa, transb, m, n, k, alpha, A, B, beta, C_, *, form="plain", slices=0,
                     tile=-1, stream=None, variant=0, levels=0) -> int:
    """Calls mpgemm_ex_noalloc (the _ex call with the library's static
    scratch buffer instead of a workspace); returns the status code."""
    P = PREC[prec]
    L = _lib.load()
    a, lda, sa = _mat(A, P)
    b, ldb, sb = _mat(B, P)
    c, ldc, sc = _mat(C_, P)
    o = make_opts(form, slices, tile, None, variant, levels)
    return L.mpgemm_ex_noalloc(P, transa.encode(), transb.encode(), m, n, k, _scalar(alpha, P), a, lda, sa,
                               b, ldb, sb, _scalar(beta, P), c, ldc, sc, _stream(stream), C.byref(o))


def gemm_noalloc(prec, transa, transb, m, n, k, alpha, A, B, beta, C_, **kw) -> None:
    """As gemm(), without a workspace: the split, residue and Strassen forms
    use the library's static scratch buffer; raises on error."""
    _check(gemm_noalloc_raw(prec, transa, transb, m, n, k, alpha, A, B, beta, C_, **kw), "mpgemm_ex_noalloc")


def gemm(prec, transa, transb, m, n, k, alpha, A, B, beta, C_, **kw) -> None:
    """C_ = alpha op(A) op(B) + beta C_ (in place); raises on error."""
    _check(gemm_raw(prec, transa, transb, m, n, k, alpha, A, B, beta, C_, **kw), "mpgemm")


def matmul(prec, A, B, C_=None, alpha=(1.0,), beta=(0.0,), **kw) -> torch.Tensor:
    """Row-major product: C_ = alpha A B + beta C_ for A (P, m, k), B (P, k, n)
    and C_ (P, m, n), each plane row-major with unit stride along a row;
    returns C_ (allocated when None, which requires beta = 0: C_ is not read).

    A row-major plane is the column-major plane of its transpose, so this is
    the column-major call C^T = B^T A^T on the same buffers (m and n
    swapped, B first).  Each product is therefore MUL(b_lj, a_il): bitwise
    the canonical chain for DD, whose multiplication is symmetric, and for
    TD and QD the canonical chain of the transposed problem (within the same
    error bound).  Keyword arguments as for gemm."""
    P = PREC[prec]
    if A.dim() != 3 or B.dim() != 3 or A.shape[0] != P or B.shape[0] != P:
        raise ValueError(f"expected A (P={P}, m, k) and B (P={P}, k, n)")
    m, k = A.shape[1], A.shape[2]
    if B.shape[1] != k:
        raise ValueError(f"inner dimensions differ: A has k = {k}, B has {B.shape[1]} rows")
    n = B.shape[2]
    if C_ is None:
        if any(float(x) != 0.0 for x in beta):
            raise ValueError("beta != 0 needs C_")
        C_ = torch.empty((P, m, n), dtype=torch.float64, device=A.device)
    elif C_.dim() != 3 or tuple(C_.shape) != (P, m, n):
        raise ValueError(f"expected C_ of shape {(P, m, n)}, got {tuple(C_.shape)}")
    gemm(prec, "N", "N", n, m, k, alpha, B, A, beta, C_, **kw)
    return C_


def vec_raw(prec, op, x, y, r, n=None, stream=None) -> int:
    P = PREC[prec]
    L = _lib.load()
    n = x.shape[-1] if n is None else n
    xs = x.stride(0) if P > 1 else n
    ys = y.stride(0) if P > 1 else n
    rs = r.stride(0) if P > 1 else n
    fn = getattr(L, f"mp_vec_{_NAME[P]}_{op}")
    return fn(n, C.c_void_p(x.data_ptr()), xs, C.c_void_p(y.data_ptr()), ys, C.c_void_p(r.data_ptr()),
              rs, _stream(stream))


def vec(prec, op, x, y, r, n=None, stream=None) -> None:
    """r = x op y element-wise; x, y, r are (P, n) float64 CUDA tensors; op is
    "add" or "mul", and for TD also "add_acc" (Algorithm 3) or "mulq"."""
    _check(vec_raw(prec, op, x, y, r, n, stream), "mp_vec")


def split_layout(prec, m, n, k, slices=0, tile=-1) -> dict:
    L = _lib.load()
    offs = [C.c_size_t() for _ in range(5)]
    dims = [C.c_int64() for _ in range(3)]
    rc = L.mpgemm_split_layout(PREC[prec], m, n, k, slices, tile, *[C.byref(o) for o in offs],
                               *[C.byref(d) for d in dims])
    _check(rc, "mpgemm_split_layout")
    keys = ["E", "F", "DA", "DB", "S"]
    out = {k_: o.value for k_, o in zip(keys, offs)}
    out.update(Mp=dims[0].value, Np=dims[1].value, Kp=dims[2].value)
    return out


def split_stages(prec, last, transa, transb, m, n, k, alpha, A, B, beta, C_, *, slices=0, tile=-1,
                 workspace=None, stream=None) -> None:
    P = PREC[prec]
    L = _lib.load()
    a, lda, sa = _mat(A, P)
    b, ldb, sb = _mat(B, P)
    c, ldc, sc = _mat(C_, P)
    o = make_opts("split", slices, tile, workspace)
    rc = L.mpgemm_split_stages(P, last, transa.encode(), transb.encode(), m, n, k, _scalar(alpha, P),
                               a, lda, sa, b, ldb, sb, _scalar(beta, P), c, ldc, sc, _stream(stream),
                               C.byref(o))
    _check(rc, "mpgemm_split_stages")


def _problem_array(P, problems):
    arr = (_lib.Problem * max(len(problems), 1))()
    keep = []
    for q, pr in enumerate(problems):
        x = arr[q]
        x.transa = pr.get("transa", "N").encode()
        x.transb = pr.get("transb", "N").encode()
        x.m, x.n, x.k = pr["m"], pr["n"], pr["k"]
        al = list(pr["alpha"]) + [0.0] * 4
        be = list(pr["beta"]) + [0.0] * 4
        x.alpha = (C.c_double * 4)(*al[:4])
        x.beta = (C.c_double * 4)(*be[:4])
        a, x.lda, x.a_plane_stride = _mat(pr["A"], P)
        b, x.ldb, x.b_plane_stride = _mat(pr["B"], P)
        c, x.ldc, x.c_plane_stride = _mat(pr["C"], P)
        x.A, x.B, x.C = a, b, c
        keep.append((pr["A"], pr["B"], pr["C"]))
    return arr, keep


class BatchPlan:
    """Many GEMMs of one precision, replayed from a captured hipGraph (run)
    or launched directly (launch): the plain part in one persistent launch,
    the residue part (form "crt", or "auto" with slices > 0) in four
    launches per chunk."""

    def __init__(self, prec, problems, tile=-1, stream=None, form="plain", slices=0, chunk_bytes=0):
        """problems: sequence of dicts with keys transa, transb, m, n, k, alpha,
        A, B, beta, C (tensors as for gemm()); chunk_bytes bounds the residue
        part's workspace per chunk (0: the library's default)."""
        self.P = PREC[prec]
        L = _lib.load()
        arr, self._keep = _problem_array(self.P, problems)
        opts = make_opts(form, slices, tile, None)
        opts.workspace_bytes = int(chunk_bytes)
        h = C.c_void_p()
        rc = L.mpgemm_batch_plan_create(self.P, len(problems), arr, C.byref(opts), _stream(stream),
                                        C.byref(h))
        _check(rc, "mpgemm_batch_plan_create")
        self._h = h

    def run(self, stream=None):
        _check(_lib.load().mpgemm_batch_plan_run(self._h, _stream(stream)), "batch run")

    def launch(self, stream=None):
        _check(_lib.load().mpgemm_batch_plan_launch(self._h, _stream(stream)), "batch launch")

    def info(self):
        t, g, c = C.c_int64(), C.c_int(), C.c_int()
        L = _lib.load()
        _check(L.mpgemm_batch_plan_info(self._h, C.byref(t), C.byref(g), C.byref(c)), "info")
        rp, mo, ch, wb = C.c_int64(), C.c_int(), C.c_int(), C.c_size_t()
        _check(L.mpgemm_batch_plan_residue_info(self._h, C.byref(rp), C.byref(mo), C.byref(ch), C.byref(wb)),
               "residue info")
        return {"tiles": t.value, "grid": g.value, "tile_cfg": c.value, "residue_problems": rp.value,
                "moduli": mo.value, "chunks": ch.value, "residue_workspace": wb.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().mpgemm_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grouped_raw(prec, problems, tile=-1, stream=None, arr=None, form="plain", slices=0) -> int:
    """Calls mpgemm_{dd,td,qd}_grouped on `problems` (dicts as for
    BatchPlan); `arr` may pass a prebuilt problem array (from
    problem_array) so that repeated calls present the same array."""
    P = PREC[prec]
    if arr is None:
        arr, _keep = _problem_array(P, problems)
    opts = make_opts(form, slices, tile, None)
    return getattr(_lib.load(), f"mpgemm_{_NAME[P]}_grouped")(len(problems), arr, C.byref(opts), _stream(stream))


def grouped(prec, problems, tile=-1, stream=None, arr=None, form="plain", slices=0) -> None:
    """All problems as one batched plan (cached by the library per problem
    array, form, slices and tile); raises on error."""
    _check(grouped_raw(prec, problems, tile, stream, arr, form, slices), "mpgemm_grouped")


def problem_array(prec, problems):
    """The ctypes problem array for grouped calls (keep the tensors alive)."""
    arr, _keep = _problem_array(PREC[prec], problems)
    return arr


def autotune(prec, form, m, n, k, slices=0, stream=None) -> int:
    best = C.c_int(-1)
    f = FORMS[form] if isinstance(form, str) else int(form)
    _check(_lib.load().mpgemm_autotune(PREC[prec], f, m, n, k, slices, _stream(stream), C.byref(best)),
           "mpgemm_autotune")
    return best.value


def batch_autotune(prec, problems, stream=None) -> int:
    """Time every tile configuration of the batched form on these problems
    (their C buffers are overwritten) and record the fastest."""
    P = PREC[prec]
    arr, keep = _problem_array(P, problems)
    best = C.c_int(-1)
    _check(_lib.load().mpgemm_batch_autotune(P, len(problems), arr, _stream(stream), C.byref(best)),
           "mpgemm_batch_autotune")
    return best.value


def autotune_set(prec, form, m, n, k, tile) -> None:
    f = FORMS[form] if isinstance(form, str) else int(form)
    _check(_lib.load().mpgemm_autotune_set(PREC[prec], f, m, n, k, tile), "autotune_set")


def autotune_save(path: str) -> None:
    _check(_lib.load().mpgemm_autotune_save(path.encode()), "autotune_save")


def autotune_load(path: str) -> None:
    _check(_lib.load().mpgemm_autotune_load(path.encode()), "autotune_load")


FORMS_ALL = dict(FORMS, batched=3)


def num_configs(prec, form) -> int:
    f = FORMS_ALL[form] if isinstance(form, str) else int(form)
    return int(_lib.load().mpgemm_num_configs(PREC[prec], f))


def tune_slices(prec, transa, transb, m, n, k, A, B, target=1.0, smin=None, smax=40, stream=None):
    """Smallest slice count whose split result on a block of rows stays within
    target * k * u * (|A||B|)_ij of the plain result; returns (s, ratio)."""
    P = PREC[prec]
    smin = DEFAULT_SLICES[P] - 4 if smin is None else smin
    a, lda, sa = _mat(A, P)
    b, ldb, sb = _mat(B, P)
    s = C.c_int()
    r = C.c_double()
    rc = _lib.load().mpgemm_tune_slices(P, transa.encode(), transb.encode(), m, n, k, a, lda, sa, b, ldb,
                                        sb, float(target), int(smin), int(smax), _stream(stream),
                                        C.byref(s), C.byref(r))
    _check(rc, "mpgemm_tune_slices")
    return s.value, r.value


def axpy(prec, alpha, x, y, n=None, stream=None) -> None:
    """y = alpha x + y element-wise (mp_axpy_*); x, y are (P, n) CUDA tensors."""
    P = PREC[prec]
    n = x.shape[-1] if n is None else n
    rc = getattr(_lib.load(), f"mp_axpy_{_NAME[P]}")(n, _scalar(alpha, P), C.c_void_p(x.data_ptr()),
                                                     x.stride(0), C.c_void_p(y.data_ptr()), y.stride(0),
                                                     _stream(stream))
    _check(rc, "mp_axpy")


def dot_workspace(prec, n, device=None) -> torch.Tensor:
    nbytes = int(_lib.load().mp_dot_workspace_bytes(PREC[prec], n))
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device or "cuda")


def dot_raw(prec, x, y, result, workspace=None, n=None, stream=None) -> int:
    P = PREC[prec]
    n = x.shape[-1] if n is None else n
    if workspace is not None:
        ws = workspace
    else:
        # a temporary used by kernels queued on `stream`: allocated on that
        # stream, so the caching allocator does not hand it out again before
        # they end
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        with torch.cuda.stream(s):
            ws = dot_workspace(prec, n, x.device)
    return getattr(_lib.load(), f"mp_dot_{_NAME[P]}")(
        n, C.c_void_p(x.data_ptr()), x.stride(0), C.c_void_p(y.data_ptr()), y.stride(0),
        C.c_void_p(result.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
        _stream(stream))


def dot(prec, x, y, result, workspace=None, n=None, stream=None) -> None:
    """result (P-element CUDA tensor) = x . y in the fixed 64-ary tree order
    (mp_dot_*); x, y are (P, n) CUDA tensors."""
    _check(dot_raw(prec, x, y, result, workspace, n, stream), "mp_dot")


def gemv_raw(prec, trans, m, n, alpha, A, x, beta, y, stream=None) -> int:
    P = PREC[prec]
    a, lda, sa = _mat(A, P)
    return getattr(_lib.load(), f"mp_gemv_{_NAME[P]}")(
        trans.encode(), m, n, _scalar(alpha, P), a, lda, sa, C.c_void_p(x.data_ptr()), x.stride(0),
        _scalar(beta, P), C.c_void_p(y.data_ptr()), y.stride(0), _stream(stream))


def gemv(prec, trans, m, n, alpha, A, x, beta, y, stream=None) -> None:
    """y = alpha op(A) x + beta y (mp_gemv_*): A a (P, n, lda) component-plane
    m x n matrix, x and y (P, len) CUDA tensors."""
    _check(gemv_raw(prec, trans, m, n, alpha, A, x, beta, y, stream), "mp_gemv")


PROBES = {"fp64_fma": 0, "fp64_add": 1, "fp64_mul": 2, "int8_mfma": 3, "hbm_copy": 4}


def probe_peak(which, stream=None) -> float:
    """Measured throughput of the GPU: flops/s for "fp64_fma", operations/s for
    "fp64_add", "fp64_mul" and "int8_mfma", bytes/s for "hbm_copy"
    (mpgemm_probe_peak)."""
    r = C.c_double()
    _check(_lib.load().mpgemm_probe_peak(PROBES[which], _stream(stream), C.byref(r)), "mpgemm_probe_peak")
    return r.value


def version() -> str:
    return _lib.load().mpgemm_version().decode()
