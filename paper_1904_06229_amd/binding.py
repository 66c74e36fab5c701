"""Python binding of libperm.so: argument marshalling only.

Every function here has the name of the C entry point it calls (see
``include/perm.h``) and does nothing but check Python-side arguments, take
device pointers and the current HIP stream from torch tensors, and call the
library through ctypes.  Every step of the computation runs in the library's
HIP kernels; there is no fallback.  If ``libperm.so`` has not been built the
import fails with an error that says so.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libperm.so")

PERM_OK, PERM_EINVAL, PERM_ERANGE, PERM_ENONFINITE, PERM_ENOMEM, PERM_EHIP, PERM_ENOTIMPL = range(7)
PERM_FP64_DD, PERM_FP64, PERM_SPLIT_F32 = 0, 1, 2
PERM_DT_REAL, PERM_DT_COMPLEX, PERM_DT_INT01 = 0, 1, 2
PRECISIONS = {"dd": PERM_FP64_DD, "fp64": PERM_FP64, "split": PERM_SPLIT_F32}


class perm_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("log2_chunk", ctypes.c_int32),
                ("drift_check", ctypes.c_int32), ("no_row_scaling", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("partials_cap", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("partials_out", ctypes.c_void_p)]


class perm_result(ctypes.Structure):
    _fields_ = [("re_hi", ctypes.c_double), ("re_lo", ctypes.c_double),
                ("im_hi", ctypes.c_double), ("im_lo", ctypes.c_double),
                ("int_lo", ctypes.c_uint64), ("int_hi", ctypes.c_int64),
                ("max_drift", ctypes.c_double), ("terms", ctypes.c_uint64),
                ("chunks", ctypes.c_uint64), ("log2_chunk", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("kernel_ms", ctypes.c_float),
                ("total_ms", ctypes.c_float), ("walk_variant", ctypes.c_int32),
                ("col0_nonzeros", ctypes.c_int32), ("parts", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class perm_plan_info(ctypes.Structure):
    _fields_ = [("log2_chunk", ctypes.c_int32), ("head_start", ctypes.c_uint64),
                ("head_count", ctypes.c_uint64), ("body_first_chunk", ctypes.c_uint64),
                ("body_chunks", ctypes.c_uint64), ("tail_start", ctypes.c_uint64),
                ("tail_count", ctypes.c_uint64), ("body_tasks", ctypes.c_uint64)]


# Every symbol include/perm.h declares, with its ctypes signature.
_vp, _i, _u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
SIGNATURES = {
    "perm_real": ([_vp, _i, _i, ctypes.POINTER(perm_opts), ctypes.POINTER(perm_result), _vp], _i),
    "perm_complex": ([_vp, _i, _i, ctypes.POINTER(perm_opts), ctypes.POINTER(perm_result), _vp], _i),
    "perm_int01": ([_vp, _i, _i, ctypes.POINTER(perm_opts), ctypes.POINTER(perm_result), _vp], _i),
    "perm_partial": ([_i, _vp, _i, _i, _u64, _u64, ctypes.POINTER(perm_opts),
                      ctypes.POINTER(perm_result), _vp], _i),
    "perm_partial_noalloc": ([_i, _vp, _i, _i, _u64, _u64, ctypes.POINTER(perm_opts),
                              ctypes.POINTER(perm_result), _vp], _i),
    "perm_batched": ([_vp, _vp, _vp, _i, _i, ctypes.POINTER(perm_opts), _vp, _vp, _vp], _i),
    "perm_sparse": ([_i, _vp, _i, _i, _i, _u64, ctypes.POINTER(perm_opts),
                     ctypes.POINTER(perm_result), _vp], _i),
    "perm_sparse_partial": ([_i, _vp, _i, _i, _i, _u64, _u64, _u64, ctypes.POINTER(perm_opts),
                             ctypes.POINTER(perm_result), _vp], _i),
    "perm_sparse_partition": ([_i, _vp, _i, _i, _i, _u64, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64),
                               _vp], _i),
    "perm_band": ([_i, _vp, _vp, _vp, _i, _i, ctypes.POINTER(perm_opts), _vp, _vp, _vp], _i),
    "perm_repeated": ([_i, _vp, _i, _i, _i, ctypes.POINTER(ctypes.c_int32),
                       ctypes.POINTER(perm_opts), ctypes.POINTER(perm_result), _vp], _i),
    "perm_repeated_partial": ([_i, _vp, _i, _i, _i, ctypes.POINTER(ctypes.c_int32), _u64, _u64,
                               ctypes.POINTER(perm_opts), ctypes.POINTER(perm_result), _vp], _i),
    "perm_combine": ([_i, _i, ctypes.POINTER(perm_result), _i, ctypes.POINTER(perm_result)], _i),
    "perm_autotune": ([_i, _i, _i, ctypes.c_char_p, _vp], _i),
    "perm_plan": ([_i, _u64, _u64, _i, _i, ctypes.POINTER(perm_plan_info)], _i),
    "perm_int01_bound": ([ctypes.POINTER(ctypes.c_int32), _i], ctypes.c_double),
    "perm_strerror": ([_i], ctypes.c_char_p),
    "perm_last_error": ([], ctypes.c_char_p),
    "perm_version": ([], ctypes.c_char_p),
    "perm_release": ([], None),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python -m paper_1904_06229_amd.build, "
            "or __graft_entry__.build()); there is no non-GPU fallback")
    # torch first: the library must bind to the HIP runtime torch has loaded
    # (torch ships its own copy; loaded the other way round, the process would
    # hold two runtimes and the library's would see no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


class PermError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.perm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.perm_strerror(status).decode()} ({status}): {msg}")


@dataclass
class Result:
    """A permanent (or partial sum) as returned by the library."""

    re_hi: float
    re_lo: float
    im_hi: float
    im_lo: float
    exact: int | None
    max_drift: float
    terms: int
    chunks: int
    log2_chunk: int
    blocks: int
    kernel_ms: float
    total_ms: float
    walk_variant: int = 0
    col0_nonzeros: int = 0
    parts: int = 0

    @property
    def value(self):
        if self.exact is not None:
            return self.exact
        if self.im_hi != 0.0 or self.im_lo != 0.0:
            return complex(self.re_hi + self.re_lo, self.im_hi + self.im_lo)
        return self.re_hi + self.re_lo


def _result(r: perm_result, exact: bool) -> Result:
    ex = None
    if exact:
        v = (r.int_lo & ((1 << 64) - 1)) | ((r.int_hi & ((1 << 64) - 1)) << 64)
        ex = v - (1 << 128) if v >= (1 << 127) else v
    return Result(r.re_hi, r.re_lo, r.im_hi, r.im_lo, ex, r.max_drift, r.terms, r.chunks,
                  r.log2_chunk, r.blocks, r.kernel_ms, r.total_ms, r.walk_variant,
                  r.col0_nonzeros, r.parts)


def make_opts(precision="dd", log2_chunk=0, drift_check=False, row_scaling=True, blocks=0,
              use_graph=False, partials=None) -> perm_opts:
    """partials: an optional float64 device tensor for the partial-sum records
    (5 doubles each; its size sets partials_cap)."""
    o = perm_opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.log2_chunk = int(log2_chunk)
    o.drift_check = 1 if drift_check else 0
    o.no_row_scaling = 0 if row_scaling else 1
    o.blocks = int(blocks)
    o.use_graph = 1 if use_graph else 0
    if partials is not None:
        import torch
        if partials.dtype != torch.float64 or not partials.is_contiguous() \
                or partials.device.type != "cuda":
            raise TypeError("partials must be a contiguous float64 device tensor")
        o.partials_out = partials.data_ptr()
        o.partials_cap = min(partials.numel() // 5, 2 ** 31 - 1)
    return o


def _stream_handle(stream):
    """The hipStream_t to enqueue on.  When it is not torch's current stream,
    it first waits (on the device) for the work already on the current one,
    so that tensors produced there -- the caller's, or a column-major copy
    made here -- are complete before the library reads them."""
    import torch
    if stream is None:
        # torch's current stream as a raw handle, without building a Stream object
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return ctypes.c_void_p(raw(torch.cuda.current_device()))
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cur = torch.cuda.current_stream()
    if stream != cur:
        stream.wait_stream(cur)
    return ctypes.c_void_p(stream.cuda_stream)


def _opts_arg(opts):
    """A perm_opts for the given keyword options, or None (NULL: the defaults)."""
    return ctypes.byref(make_opts(**opts)) if opts else None


def _matrix(A, dtype_name):
    """(pointer, n, ld) of a square device tensor, viewed column-major.

    A row-major tensor is passed as the column-major array of its transpose;
    per(A^T) = per(A), so no copy is needed.
    """
    import torch
    if not isinstance(A, torch.Tensor) or A.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) torch tensor")
    want = {"real": torch.float64, "complex": torch.complex128, "int01": torch.uint8}[dtype_name]
    if A.dtype != want:
        raise TypeError(f"expected dtype {want}, got {A.dtype}")
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    n = A.shape[0]
    if n == 0:
        return ctypes.c_void_p(A.data_ptr() or 0), 0, 1
    s0, s1 = A.stride()
    if s1 == 1 and s0 >= n:
        ld = s0
    elif s0 == 1 and s1 >= n:
        ld = s1
    elif n == 1:
        ld = 1
    else:
        raise ValueError("matrix must have unit stride along one dimension")
    return ctypes.c_void_p(A.data_ptr()), n, ld


def _check(st, where):
    if st != PERM_OK:
        raise PermError(st, where)


def perm_real(A, stream=None, **opts) -> Result:
    p, n, ld = _matrix(A, "real")
    r = perm_result()
    _check(_lib.perm_real(p, n, ld, _opts_arg(opts), ctypes.byref(r), _stream_handle(stream)),
           "perm_real")
    return _result(r, False)


def perm_complex(A, stream=None, **opts) -> Result:
    p, n, ld = _matrix(A, "complex")
    r = perm_result()
    _check(_lib.perm_complex(p, n, ld, _opts_arg(opts), ctypes.byref(r), _stream_handle(stream)),
           "perm_complex")
    return _result(r, False)


def perm_int01(A, stream=None, **opts) -> Result:
    p, n, ld = _matrix(A, "int01")
    r = perm_result()
    _check(_lib.perm_int01(p, n, ld, _opts_arg(opts), ctypes.byref(r), _stream_handle(stream)),
           "perm_int01")
    return _result(r, True)


def _partial_call(fn, name, A, start, count, stream, opts) -> Result:
    import torch
    kind = {torch.float64: "real", torch.complex128: "complex", torch.uint8: "int01"}[A.dtype]
    dt = {"real": PERM_DT_REAL, "complex": PERM_DT_COMPLEX, "int01": PERM_DT_INT01}[kind]
    if A.dim() == 2 and A.shape[0] > 1 and A.stride(0) != 1:
        A = A.t().contiguous().t()
    p, n, ld = _matrix(A, kind)
    o, r = make_opts(**opts), perm_result()
    _check(fn(dt, p, n, ld, int(start), int(count), ctypes.byref(o), ctypes.byref(r),
              _stream_handle(stream)), name)
    return _result(r, kind == "int01")


def perm_partial(A, start: int, count: int, stream=None, **opts) -> Result:
    """Partial sum of the terms of A itself (entry A[i, j] in row i, column j).

    Unlike the full permanent, a partial sum changes under transposition, so
    the library must see A column-major: a row-major tensor is copied to
    column-major storage first (pass A.t().contiguous().t() to avoid it).
    """
    return _partial_call(_lib.perm_partial, "perm_partial", A, start, count, stream, opts)


def perm_partial_noalloc(A, start: int, count: int, stream=None, **opts) -> Result:
    """perm_partial on the library's fixed device array (the library allocates
    nothing; calls on one device must not overlap).  A column-major tensor
    avoids the copy a row-major one gets here."""
    return _partial_call(_lib.perm_partial_noalloc, "perm_partial_noalloc", A, start, count,
                         stream, opts)


def _to_struct(res: Result) -> perm_result:
    r = perm_result()
    r.re_hi, r.re_lo, r.im_hi, r.im_lo = res.re_hi, res.re_lo, res.im_hi, res.im_lo
    if res.exact is not None:
        v = res.exact & ((1 << 128) - 1)
        r.int_lo = v & ((1 << 64) - 1)
        hi = v >> 64
        r.int_hi = hi - (1 << 64) if hi >= (1 << 63) else hi
    r.max_drift, r.terms, r.chunks = res.max_drift, res.terms, res.chunks
    r.log2_chunk, r.blocks = res.log2_chunk, res.blocks
    r.kernel_ms, r.total_ms = res.kernel_ms, res.total_ms
    return r


def perm_combine(kind: str, n: int, parts) -> Result:
    """per(A) = 2(-1)^n sum_k S_k from perm_partial results covering the whole
    range once, added in the given order (App. A, permanent).  kind: "real",
    "complex" or "int01"."""
    dt = {"real": PERM_DT_REAL, "complex": PERM_DT_COMPLEX, "int01": PERM_DT_INT01}[kind]
    parts = list(parts)
    arr = (perm_result * max(len(parts), 1))(*[_to_struct(p) for p in parts])
    r = perm_result()
    _check(_lib.perm_combine(dt, int(n), arr, len(parts), ctypes.byref(r)), "perm_combine")
    return _result(r, kind == "int01")


def _distinct_columns(C, mult):
    """(dtype code, pointer, n, R, ld, multiplicity array) for an n x R device
    tensor of distinct columns; a row-major tensor is copied to column-major
    (C is not square, so the transpose is not an option)."""
    import torch
    if not isinstance(C, torch.Tensor) or C.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if C.dtype == torch.float64:
        dt = PERM_DT_REAL
    elif C.dtype == torch.complex128:
        dt = PERM_DT_COMPLEX
    else:
        raise TypeError(f"expected float64 or complex128, got {C.dtype}")
    if C.dim() != 2:
        raise ValueError("C must be n x R")
    n, R = C.shape
    if len(mult) != R:
        raise ValueError("one multiplicity per column of C")
    if n > 1 and C.stride(0) != 1:
        C = C.t().contiguous().t()
    ld = C.stride(1) if R > 1 else max(n, 1)
    m = (ctypes.c_int32 * max(R, 1))(*[int(x) for x in mult])
    return dt, ctypes.c_void_p(C.data_ptr()), n, R, max(ld, n, 1), m, C


def perm_repeated(C, mult, stream=None, **opts) -> Result:
    """per(A), A having column k of C repeated mult[k] times (Eq. ryser2)."""
    dt, p, n, R, ld, m, keep = _distinct_columns(C, mult)
    o, r = make_opts(**opts), perm_result()
    _check(_lib.perm_repeated(dt, p, n, R, ld, m, ctypes.byref(o), ctypes.byref(r),
                              _stream_handle(stream)), "perm_repeated")
    return _result(r, False)


def perm_repeated_partial(C, mult, start: int, count: int, stream=None, **opts) -> Result:
    """Raw Eq. ryser2 sum (no (-1)^n) over reflected mixed-radix Gray indices [start, start+count)."""
    dt, p, n, R, ld, m, keep = _distinct_columns(C, mult)
    o, r = make_opts(**opts), perm_result()
    _check(_lib.perm_repeated_partial(dt, p, n, R, ld, m, int(start), int(count), ctypes.byref(o),
                                      ctypes.byref(r), _stream_handle(stream)),
           "perm_repeated_partial")
    return _result(r, False)


def _square_cm(A):
    """(dtype code, pointer, n, ld, tensor) of a square device matrix seen
    column-major; a row-major tensor is copied (a partial sum or a partition
    is not invariant under transposition)."""
    import torch
    if not isinstance(A, torch.Tensor) or A.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) torch tensor")
    dt = {torch.float64: PERM_DT_REAL, torch.complex128: PERM_DT_COMPLEX,
          torch.uint8: PERM_DT_INT01}.get(A.dtype)
    if dt is None:
        raise TypeError(f"expected float64, complex128 or uint8, got {A.dtype}")
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    n = A.shape[0]
    if n > 1 and A.stride(0) != 1:
        A = A.t().contiguous().t()
    ld = A.stride(1) if n > 1 else max(n, 1)
    return dt, ctypes.c_void_p(A.data_ptr()), n, max(ld, n, 1), A


def perm_sparse(A, trials: int = 1, seed: int = 0, stream=None, **opts) -> Result:
    """per(A) by App. B's restricted Ryser sum (exact for uint8 input within its bound)."""
    dt, p, n, ld, keep = _square_cm(A)
    o, r = make_opts(**opts), perm_result()
    _check(_lib.perm_sparse(dt, p, n, ld, int(trials), int(seed), ctypes.byref(o), ctypes.byref(r),
                            _stream_handle(stream)), "perm_sparse")
    return _result(r, dt == PERM_DT_INT01)


def perm_sparse_partial(A, start: int, count: int, trials: int = 1, seed: int = 0, stream=None,
                        **opts) -> Result:
    """Raw App. B sum (no (-1)^n) over Gray indices [start, start+count) of its enumeration."""
    dt, p, n, ld, keep = _square_cm(A)
    o, r = make_opts(**opts), perm_result()
    _check(_lib.perm_sparse_partial(dt, p, n, ld, int(trials), int(seed), int(start), int(count),
                                    ctypes.byref(o), ctypes.byref(r), _stream_handle(stream)),
           "perm_sparse_partial")
    return _result(r, dt == PERM_DT_INT01)


def perm_sparse_partition(A, trials: int = 1, seed: int = 0, stream=None):
    """(block index of every column or -1, number of blocks, number of column sets)."""
    dt, p, n, ld, keep = _square_cm(A)
    blk = (ctypes.c_int32 * n)()
    nb, terms = ctypes.c_int32(), ctypes.c_uint64()
    _check(_lib.perm_sparse_partition(dt, p, n, ld, int(trials), int(seed), blk, ctypes.byref(nb),
                                      ctypes.byref(terms), _stream_handle(stream)),
           "perm_sparse_partition")
    return [int(x) for x in blk], nb.value, terms.value


def _host_ints(seq, dtype):
    """A C-contiguous host array of `dtype` holding `seq` (zero-copy for a
    matching numpy array) and its address, for the size/offset arguments.
    Values outside `dtype` raise instead of wrapping."""
    import numpy as np
    raw = np.asarray(seq)
    if raw.ndim != 1:
        raise ValueError("sizes and offsets must be one-dimensional")
    if raw.size and raw.dtype.kind not in "iu":
        raise TypeError("sizes and offsets must be integers")
    info = np.iinfo(dtype)
    if raw.size and (int(raw.min()) < info.min or int(raw.max()) > info.max):
        raise ValueError(f"a size or offset does not fit {np.dtype(dtype).name}")
    arr = np.ascontiguousarray(raw.astype(dtype, copy=False))
    if arr.size == 0:
        arr = np.zeros(1, dtype=dtype)
    return arr, ctypes.c_void_p(arr.ctypes.data)


def perm_band(A_packed, sizes, offsets, k: int, is_complex: bool, out, status=None, stream=None,
              **opts) -> None:
    """Band permanents (App. C) of the matrices packed in ``A_packed``; results in ``out``."""
    import torch
    count = len(sizes)
    if len(offsets) != count:
        raise ValueError("sizes and offsets differ in length")
    n_keep, n_arr = _host_ints(sizes, "int32")
    o_keep, o_arr = _host_ints(offsets, "int64")
    o = make_opts(**opts)
    if A_packed.dtype != torch.float64 or out.dtype != torch.float64:
        raise TypeError("A_packed and out must be float64 (complex data as interleaved pairs)")
    if out.numel() < 4 * count:
        raise ValueError("out needs 4 doubles per matrix")
    st_ptr = ctypes.c_void_p(status.data_ptr()) if status is not None else ctypes.c_void_p(0)
    dt = PERM_DT_COMPLEX if is_complex else PERM_DT_REAL
    _check(_lib.perm_band(dt, ctypes.c_void_p(A_packed.data_ptr()), n_arr, o_arr, count, int(k),
                          ctypes.byref(o), ctypes.c_void_p(out.data_ptr()), st_ptr,
                          _stream_handle(stream)), "perm_band")


def perm_batched(A_packed, sizes, offsets, is_complex: bool, out, status=None, stream=None,
                 **opts) -> None:
    """Enqueue the batched permanents; results land in ``out`` (float64, 4 per matrix)."""
    import torch
    count = len(sizes)
    if len(offsets) != count:
        raise ValueError("sizes and offsets differ in length")
    n_keep, n_arr = _host_ints(sizes, "int32")
    o_keep, o_arr = _host_ints(offsets, "int64")
    o = make_opts(**opts)
    if A_packed.dtype != torch.float64 or out.dtype != torch.float64:
        raise TypeError("A_packed and out must be float64 (complex data as interleaved pairs)")
    if out.numel() < 4 * count:
        raise ValueError("out needs 4 doubles per matrix")
    st_ptr = ctypes.c_void_p(status.data_ptr()) if status is not None else ctypes.c_void_p(0)
    _check(_lib.perm_batched(ctypes.c_void_p(A_packed.data_ptr()), n_arr, o_arr, count,
                             1 if is_complex else 0, ctypes.byref(o),
                             ctypes.c_void_p(out.data_ptr()), st_ptr, _stream_handle(stream)),
           "perm_batched")


def perm_autotune(is_complex: bool, n_lo: int, n_hi: int, cache_path: str | None = None,
                  stream=None) -> None:
    cp = cache_path.encode() if cache_path else None
    _check(_lib.perm_autotune(1 if is_complex else 0, n_lo, n_hi, cp, _stream_handle(stream)),
           "perm_autotune")


def perm_plan(n: int, start: int, count: int, log2_chunk: int = 0, is_int01: bool = False) -> dict:
    p = perm_plan_info()
    _check(_lib.perm_plan(n, start, count, log2_chunk, 1 if is_int01 else 0, ctypes.byref(p)),
           "perm_plan")
    return {f: getattr(p, f) for f, _ in perm_plan_info._fields_}


def perm_int01_bound(degrees) -> float:
    d = (ctypes.c_int32 * max(len(degrees), 1))(*[int(x) for x in degrees])
    return _lib.perm_int01_bound(d, len(degrees))


def perm_strerror(status: int) -> str:
    return _lib.perm_strerror(status).decode()


def perm_last_error() -> str:
    return _lib.perm_last_error().decode()


def perm_version() -> str:
    return _lib.perm_version().decode()


def perm_release() -> None:
    _lib.perm_release()
