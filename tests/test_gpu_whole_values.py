"""GPU: whole permanents at the two largest floating-point sizes, pinned to
values the oracle fixes.

The 40 x 40 complex and 48 x 48 real workloads have 2^39 and 2^47 Gray
terms, far beyond the oracle's reach as a whole.  Their whole values are
pinned here by structure and by the mathematics:

* block-diagonal matrices: per(X (+) Y) = per(X) per(Y) (expand the
  definition, Sec. I, Eq. per: a permutation with a nonzero product maps each
  block's rows onto that block's columns).  The 40 x 40 matrix keeps the two
  20 x 20 diagonal blocks of the benchmark's Haar block; the 48 x 48 matrix the
  two 24 x 24 diagonal blocks of the benchmark's Gaussian matrix.  Each block's
  permanent comes from the oracle's long-double Ryser sum (Eq. ryser), and the
  product is formed exactly.  The GPU sees a 40 x 40 (48 x 48) matrix and
  walks all of its 2^39 (2^47) terms in the benchmark's configuration: the
  same call, chunk length and grid (the 48 x 48 one as 16 perm_partial
  slices added by perm_combine, App. A permanent);
* the benchmarked 40 x 40 Haar block itself: a sub-block of a unitary matrix
  has operator norm at most 1, and |per A| <= ||A||^n, so |per| <= 1; and
  the plain FP64 sum must agree with the double-double sum to the FP64 bar.

Tolerance: 1e-10 relative (the FP64 bar).  Rounding of the 2^47 products
gives about 1e-13 here.
"""
import sys
from fractions import Fraction

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def B():
    from paper_1904_06229_amd import binding
    return binding


@pytest.fixture(scope="module")
def inp():
    from paper_1904_06229_amd import inputs
    return inputs


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cfrac(x):
    """(re, im) as exact Fractions of an oracle value or a library Result."""
    if hasattr(x, "re_hi"):
        return (Fraction(x.re_hi) + Fraction(x.re_lo), Fraction(x.im_hi) + Fraction(x.im_lo))
    if hasattr(x, "re"):
        return (x.re.exact, x.im.exact)
    return (x.exact, Fraction(0))


def cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def rel(got, want):
    d = (got[0] - want[0], got[1] - want[1])
    return float(((d[0] ** 2 + d[1] ** 2) / (want[0] ** 2 + want[1] ** 2))) ** 0.5


def block_diag(A, k):
    D = np.zeros_like(A)
    D[:k, :k] = A[:k, :k]
    D[k:, k:] = A[k:, k:]
    return D


@pytest.fixture(scope="module")
def c3(B, inp):
    """The 40 x 40 benchmark matrix and its whole permanent in the
    benchmark's call (perm_complex, default options, the row-major array)."""
    A = inp.haar_block(40, 1600, 20190402)
    log("40x40 Haar block: whole permanent, double-double sums")
    r = B.perm_complex(torch.from_numpy(np.ascontiguousarray(A)).to("cuda"))
    return A, r


def test_complex40_block_diagonal_whole(B, orc, inp):
    n = 40
    U = inp.haar_block(n, n * n, 20190402)
    A = block_diag(U, 20)
    want = cmul(cfrac(orc.ryser(A[:20, :20])), cfrac(orc.ryser(A[20:, 20:])))
    log("40x40 complex, 20 (+) 20 block-diagonal: whole permanent (2^39 terms)")
    got = B.perm_complex(torch.from_numpy(np.ascontiguousarray(A)).to("cuda"))
    assert got.terms == 1 << (n - 1)
    e = rel(cfrac(got), want)
    log(f"  rel err vs product of oracle blocks {e:.2e}")
    assert e < TOL


def test_complex40_unitary_bound_and_fp64_agreement(B, c3):
    A, dd = c3
    v = complex(dd.re_hi + dd.re_lo, dd.im_hi + dd.im_lo)
    assert 0.0 < abs(v) <= 1.0
    log("40x40 Haar block: whole permanent, plain FP64 sums")
    plain = B.perm_complex(torch.from_numpy(np.ascontiguousarray(A)).to("cuda"), precision="fp64")
    e = rel(cfrac(plain), cfrac(dd))
    log(f"  |per| = {abs(v):.4e}; FP64 vs double-double sums: rel diff {e:.2e}")
    assert e < TOL


def test_complex40_split_precision_reported(B, c3):
    """FP32 products of FP64 row sums, double-double sums: the error against
    the FP64 kernel is reported, not held to 1e-10 (FP32 rounding of the 40
    factors of every term, amplified by the cancellation among the terms)."""
    A, dd = c3
    log("40x40 Haar block: whole permanent, FP32 products")
    sp = B.perm_complex(torch.from_numpy(np.ascontiguousarray(A)).to("cuda"), precision="split")
    e = rel(cfrac(sp), cfrac(dd))
    log(f"  FP32-product vs FP64 kernel: rel diff {e:.2e}")
    assert e < 1e-2


def test_complex40_whole_equals_split_partials(B, c3):
    """The whole 40 x 40 permanent (on A^T) against three perm_partial ranges
    of A's Gray enumeration with unaligned cuts, added by perm_combine.  The
    two chunkings start their walks at different terms, so their row sums
    carry different rounding, which the cancellation in the sum amplifies
    (about 4e-12 here); the bar is the FP64 one."""
    A, whole = c3
    n = 40
    T = 1 << (n - 1)
    log("40x40 complex: three partial ranges")
    cuts = [0, T // 3 + 12345, (2 * T) // 3 - 77, T]
    dA = torch.from_numpy(np.asfortranarray(A)).to("cuda")
    parts = [B.perm_partial(dA, a, b - a) for a, b in zip(cuts[:-1], cuts[1:])]
    per = B.perm_combine("complex", n, parts)
    e = rel(cfrac(whole), cfrac(per))
    log(f"  per = {whole.value:.6e}, rel diff to the combined ranges {e:.2e}")
    assert e < TOL


@pytest.mark.timeout(1500)
def test_real48_block_diagonal_whole(B, orc, inp, capsys):
    """The 48 x 48 real path as the benchmark runs it: 16 slices of 2^43
    terms (about 25 s each on one MI355X), one progress line per slice."""
    from paper_1904_06229_amd import longrun
    n = 48
    A = block_diag(inp.real_gaussian(n, 20190403), 24)
    want = orc.ryser(A[:24, :24]).exact * orc.ryser(A[24:, 24:]).exact

    def progress(msg):
        with capsys.disabled():
            print(f"  48x48 24 (+) 24 block-diagonal: {msg}", flush=True)

    progress("16 slices of 2^43 terms")
    res, info = longrun.run_sliced(torch.from_numpy(np.asfortranarray(A)).to("cuda"),
                                   slices=16, progress=progress)
    assert res.terms == 1 << (n - 1)
    got = Fraction(res.re_hi) + Fraction(res.re_lo)
    e = abs(float((got - want) / want))
    progress(f"per = {float(got):.6e}, rel err vs product of oracle blocks {e:.2e}, "
             f"{sum(info['seconds']):.0f} s")
    assert e < TOL
