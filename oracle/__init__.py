"""CPU oracle for the matrix permanent -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it and
shares no code with it; the two meet only through the seeded inputs that
``paper_1904_06229_amd.inputs`` generates.

The arithmetic lives in ``perm_oracle.c`` (plain C, long double / exact
128-bit integers); this module only compiles it with gcc and marshals numpy
arrays through ctypes.  Routes (see the C file for the passages they follow):

* ``brute``         -- the n!-term definition (Sec. I, Eq. per), n <= 12.
* ``ryser``         -- Ryser's 2^n-subset formula (Sec. II.A, Eq. ryser) in
                       Gray order with a long-double Kahan sum (App. A).
* ``ryser_range``   -- the raw signed Ryser sum over a subset-index range.
* ``chunk_partial`` -- App. A ``subpermanent`` partial sum over a Gray-index
                       range, each term formed directly (no walk).
* ``ryser2``        -- Ryser's formula for repeated columns (Sec. II.A,
                       Eq. ryser2) from the distinct columns and their
                       multiplicities; ``ryser2_range`` is its raw sum over a
                       range of the reflected mixed-radix Gray order, and
                       ``mixed_gray`` unranks that order.
* ``sparse``        -- App. B: greedypartition, then Eq. ryser over the column
                       sets that meet every block (``sparse_range``: raw sum
                       over a range of its mixed-radix Gray order;
                       ``sparse_partition`` / ``sparse_set`` expose the
                       partition and the set of a Gray index).
* ``band``          -- the band transfer matrix of App. C (bandpermanent) for
                       matrices with a_ij = 0 when |i - j| > k.

Real results come back as :class:`Pair` (an unevaluated double pair hi + lo
holding the long-double value), complex ones as :class:`CPair`, integer ones
as Python ``int``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: Kahan summation must survive)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-std=gnu11",
             "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_uint64)
    bp = ctypes.POINTER(ctypes.c_uint8)
    i, u64 = ctypes.c_int, ctypes.c_uint64
    sig = {
        "oracle_brute_real": ([dp, i, i, dp]),
        "oracle_brute_complex": ([dp, i, i, dp]),
        "oracle_brute_int": ([bp, i, i, up]),
        "oracle_ryser_real": ([dp, i, i, i, dp]),
        "oracle_ryser_complex": ([dp, i, i, i, dp]),
        "oracle_ryser_int": ([bp, i, i, i, up]),
        "oracle_ryser_real_range": ([dp, i, i, u64, u64, i, dp]),
        "oracle_ryser_complex_range": ([dp, i, i, u64, u64, i, dp]),
        "oracle_ryser_int_range": ([bp, i, i, u64, u64, i, up]),
        "oracle_chunk_real": ([dp, i, i, u64, u64, i, dp]),
        "oracle_chunk_complex": ([dp, i, i, u64, u64, i, dp]),
        "oracle_chunk_int": ([bp, i, i, u64, u64, i, up]),
        "oracle_default_threads": ([]),
        "oracle_ryser2": ([dp, i, i, i, ctypes.POINTER(ctypes.c_int), i, i, dp]),
        "oracle_ryser2_range": ([dp, i, i, i, ctypes.POINTER(ctypes.c_int), i, u64, u64, i, dp]),
        "oracle_sparse_real": ([dp, i, i, i, i, dp, up]),
        "oracle_sparse_int": ([bp, i, i, i, up, up]),
        "oracle_sparse_range": ([dp, i, i, i, u64, u64, i, dp]),
        "oracle_sparse_range_int": ([bp, i, i, u64, u64, i, up]),
        "oracle_sparse_partition": ([dp, i, i, i, ctypes.POINTER(ctypes.c_int)]),
        "oracle_sparse_set": ([dp, i, i, i, u64, up]),
        "oracle_band_real": ([dp, i, i, i, i, dp]),
        "oracle_band_int": ([bp, i, i, i, up]),
        "oracle_mixed_gray": ([u64, i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _lib = lib
    return lib


@dataclass(frozen=True)
class Pair:
    """Real value hi + lo (both doubles)."""

    hi: float
    lo: float = 0.0

    @property
    def exact(self) -> Fraction:
        return Fraction(self.hi) + Fraction(self.lo)

    def __float__(self) -> float:
        return float(self.hi)

    def __neg__(self) -> "Pair":
        return Pair(-self.hi, -self.lo)


@dataclass(frozen=True)
class CPair:
    """Complex value (re.hi + re.lo) + i (im.hi + im.lo)."""

    re: Pair
    im: Pair

    def __complex__(self) -> complex:
        return complex(self.re.hi, self.im.hi)

    def __neg__(self) -> "CPair":
        return CPair(-self.re, -self.im)


def _words_to_int(w) -> int:
    """(low, high) 64-bit words of a value mod 2^128 -> signed Python int."""
    v = int(w[0]) | (int(w[1]) << 64)
    return v - (1 << 128) if v >= (1 << 127) else v


def _prep(A):
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    n = A.shape[0]
    if np.iscomplexobj(A):
        M = np.asfortranarray(A, dtype=np.complex128)
        kind = "complex"
    elif A.dtype == np.uint8 or A.dtype == np.bool_:
        M = np.asfortranarray(A, dtype=np.uint8)
        kind = "int"
    else:
        M = np.asfortranarray(A, dtype=np.float64)
        kind = "real"
    return M, n, kind


def _ptr(M, kind):
    if kind == "int":
        return M.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return M.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _result(kind, buf):
    if kind == "real":
        return Pair(buf[0], buf[1])
    if kind == "complex":
        return CPair(Pair(buf[0], buf[1]), Pair(buf[2], buf[3]))
    return _words_to_int(buf)


def _outbuf(kind):
    if kind == "int":
        return (ctypes.c_uint64 * 2)()
    return (ctypes.c_double * 4)()


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments")


def brute(A):
    """per(A) by the definition, all n! permutations (n <= 12)."""
    lib = _load()
    M, n, kind = _prep(A)
    out = _outbuf(kind)
    f = {"real": lib.oracle_brute_real, "complex": lib.oracle_brute_complex,
         "int": lib.oracle_brute_int}[kind]
    _check(f(_ptr(M, kind), n, max(n, 1), out), "brute")
    return _result(kind, out)


def ryser(A, threads: int = 0):
    """per(A) by Ryser's formula over all 2^n subsets (n <= 40)."""
    lib = _load()
    M, n, kind = _prep(A)
    out = _outbuf(kind)
    f = {"real": lib.oracle_ryser_real, "complex": lib.oracle_ryser_complex,
         "int": lib.oracle_ryser_int}[kind]
    _check(f(_ptr(M, kind), n, max(n, 1), threads, out), "ryser")
    return _result(kind, out)


def ryser_range(A, k0: int, count: int, threads: int = 0):
    """Raw sum over subset indices [k0, k0+count) of (-1)^|J| prod_i sum_{j in J} a_ij."""
    lib = _load()
    M, n, kind = _prep(A)
    out = _outbuf(kind)
    f = {"real": lib.oracle_ryser_real_range, "complex": lib.oracle_ryser_complex_range,
         "int": lib.oracle_ryser_int_range}[kind]
    _check(f(_ptr(M, kind), n, n, k0, count, threads, out), "ryser_range")
    return _result(kind, out)


def chunk_partial(A, g0: int, count: int, threads: int = 0):
    """App. A partial sum over Gray indices [g0, g0+count): sum (-1)^(g+1) prod_i w_i.

    For 0/1 (uint8) input the integer form with r = 2w is returned instead,
    i.e. 2^n times the App. A partial sum, exactly (mod 2^128).
    """
    lib = _load()
    M, n, kind = _prep(A)
    out = _outbuf(kind)
    f = {"real": lib.oracle_chunk_real, "complex": lib.oracle_chunk_complex,
         "int": lib.oracle_chunk_int}[kind]
    _check(f(_ptr(M, kind), n, n, g0, count, threads, out), "chunk_partial")
    return _result(kind, out)


def _prep_rep(C, mult):
    C = np.asarray(C)
    if C.ndim != 2:
        raise ValueError("C must be n x R")
    n, R = C.shape
    if len(mult) != R:
        raise ValueError("one multiplicity per column of C")
    m = (ctypes.c_int * max(R, 1))(*[int(x) for x in mult])
    if np.iscomplexobj(C):
        return np.asfortranarray(C, dtype=np.complex128), n, R, m, 1
    return np.asfortranarray(C, dtype=np.float64), n, R, m, 0


def _rep_result(cplx, out):
    if cplx:
        return CPair(Pair(out[0], out[1]), Pair(out[2], out[3]))
    return Pair(out[0], out[1])


def ryser2(C, mult, threads: int = 0):
    """per(A) by Eq. ryser2, A having column k of C repeated mult[k] times."""
    lib = _load()
    M, n, R, m, cplx = _prep_rep(C, mult)
    out = (ctypes.c_double * 4)()
    _check(lib.oracle_ryser2(M.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, R, n, m,
                             cplx, threads, out), "ryser2")
    return _rep_result(cplx, out)


def ryser2_range(C, mult, g0: int, count: int, threads: int = 0):
    """Raw Eq. ryser2 sum (no (-1)^n) over reflected mixed-radix Gray indices [g0, g0+count)."""
    lib = _load()
    M, n, R, m, cplx = _prep_rep(C, mult)
    out = (ctypes.c_double * 4)()
    _check(lib.oracle_ryser2_range(M.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, R, n,
                                   m, cplx, g0, count, threads, out), "ryser2_range")
    return _rep_result(cplx, out)


def mixed_gray(g: int, radices):
    """Digits (digit 0 fastest) of index g in the reflected mixed-radix Gray order."""
    lib = _load()
    R = len(radices)
    r = (ctypes.c_int * R)(*[int(x) for x in radices])
    f = (ctypes.c_int * R)()
    _check(lib.oracle_mixed_gray(g, R, r, f), "mixed_gray")
    return [int(x) for x in f]


def _prep_float(A):
    M, n, kind = _prep(A)
    if kind == "int":
        M = np.asfortranarray(M, dtype=np.float64)
        kind = "real"
    return M, n, 1 if kind == "complex" else 0


def sparse(A, threads: int = 0):
    """(per(A), number of column sets enumerated) by App. B's sparse Ryser sum."""
    lib = _load()
    M, n, kind = _prep(A)
    terms = ctypes.c_uint64()
    if kind == "int":
        out = (ctypes.c_uint64 * 2)()
        _check(lib.oracle_sparse_int(_ptr(M, kind), n, max(n, 1), threads, out,
                                     ctypes.byref(terms)), "sparse")
        return _words_to_int(out), terms.value
    out = (ctypes.c_double * 4)()
    cplx = 1 if kind == "complex" else 0
    _check(lib.oracle_sparse_real(_ptr(M, kind), n, max(n, 1), cplx, threads, out,
                                  ctypes.byref(terms)), "sparse")
    val = CPair(Pair(out[0], out[1]), Pair(out[2], out[3])) if cplx else Pair(out[0], out[1])
    return val, terms.value


def sparse_range_int(A, g0: int, count: int, threads: int = 0) -> int:
    """0/1 data: the raw App. B sum over Gray indices [g0, g0+count) of its
    digit order, exact modulo 2^128 (as a signed int)."""
    lib = _load()
    M, n, kind = _prep(A)
    if kind != "int":
        raise TypeError("sparse_range_int takes a 0/1 (uint8) matrix")
    out = (ctypes.c_uint64 * 2)()
    _check(lib.oracle_sparse_range_int(_ptr(M, kind), n, max(n, 1), g0, count, threads, out),
           "sparse_range_int")
    return _words_to_int(out)


def sparse_range(A, g0: int, count: int, threads: int = 0):
    """Raw App. B sum (no (-1)^n) over Gray indices [g0, g0+count) of its digit order."""
    lib = _load()
    M, n, cplx = _prep_float(A)
    out = (ctypes.c_double * 4)()
    _check(lib.oracle_sparse_range(M.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                                   max(n, 1), cplx, g0, count, threads, out), "sparse_range")
    return CPair(Pair(out[0], out[1]), Pair(out[2], out[3])) if cplx else Pair(out[0], out[1])


def sparse_partition(A):
    """Block index of every column (selection order), -1 for the columns of T."""
    lib = _load()
    M, n, cplx = _prep_float(A)
    blk = (ctypes.c_int * n)()
    nb = lib.oracle_sparse_partition(M.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                                     max(n, 1), cplx, blk)
    if nb < 0:
        raise ValueError("oracle sparse_partition: invalid arguments or a zero row")
    return [int(x) for x in blk]


def sparse_set(A, g: int) -> int:
    """Column set (bit mask) of Gray index g of the App. B enumeration."""
    lib = _load()
    M, n, cplx = _prep_float(A)
    J = ctypes.c_uint64()
    _check(lib.oracle_sparse_set(M.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, max(n, 1),
                                 cplx, g, ctypes.byref(J)), "sparse_set")
    return J.value


def band(A, k: int):
    """per(A) by the App. C transfer matrix; A must vanish outside |i - j| <= k (k <= 9)."""
    lib = _load()
    M, n, kind = _prep(A)
    if kind == "int":
        out = (ctypes.c_uint64 * 2)()
        _check(lib.oracle_band_int(_ptr(M, kind), n, max(n, 1), k, out), "band")
        return _words_to_int(out)
    out = (ctypes.c_double * 4)()
    _check(lib.oracle_band_real(_ptr(M, kind), n, max(n, 1), k, 1 if kind == "complex" else 0,
                                out), "band")
    return CPair(Pair(out[0], out[1]), Pair(out[2], out[3])) if kind == "complex" \
        else Pair(out[0], out[1])


def default_threads() -> int:
    return _load().oracle_default_threads()
