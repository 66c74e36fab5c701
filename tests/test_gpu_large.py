"""GPU parity at the full sizes the oracle cannot sum in whole.

The 48x48 real and 40x40 complex workloads have 2^47 and 2^39 terms.  Their
chunk sums are checked one by one: perm_partial over a chunk [c L, (c+1) L)
runs the same walk kernel template with the same chunk length as the full
call (L = 2^12 for both), and the oracle forms every term of that chunk
directly from its Gray code (no walk, long double), App. A.
"""
import math
import sys

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


def dev_cm(A):
    return torch.from_numpy(np.asfortranarray(A)).to("cuda")


def val(x):
    if hasattr(x, "re_hi"):
        return complex(x.re_hi + x.re_lo, x.im_hi + x.im_lo)
    if hasattr(x, "re"):
        return complex(x.re.hi + x.re.lo, x.im.hi + x.im.lo)
    return complex(x.hi + x.lo, 0.0)


def rel(a, b):
    return abs(a - b) / abs(b)


def sampled_chunks(n, L, count, seed):
    total = (1 << (n - 1)) // L
    r = np.random.default_rng(seed)
    picks = [0, total - 1] + [int(x) for x in r.integers(1, total - 1, size=count - 2)]
    return picks


def check_chunks(B, orc, A, n, L, precision, tol, picks):
    worst = 0.0
    dA = dev_cm(A)
    for c in picks:
        got = B.perm_partial(dA, c * L, L, log2_chunk=int(math.log2(L)), precision=precision)
        want = orc.chunk_partial(A, c * L, L)
        e = rel(val(got), val(want))
        worst = max(worst, e)
        assert e < tol, (c, e)
    return worst


def test_real48_sampled_chunks(B, orc, inp):
    n, L = 48, 1 << 12
    A = inp.real_gaussian(n, 20190403)
    picks = sampled_chunks(n, L, 16, 48)
    w64 = check_chunks(B, orc, A, n, L, "dd", TOL, picks)
    wsp = check_chunks(B, orc, A, n, L, "split", 1e-3, picks)
    log(f"48x48 real: 16 chunks of 2^12, worst rel err FP64 {w64:.2e}, FP32-product {wsp:.2e}")


def test_complex40_sampled_chunks(B, orc, inp):
    n, L = 40, 1 << 12
    A = inp.haar_block(n, n * n, 20190402)
    picks = sampled_chunks(n, L, 16, 40)
    w64 = check_chunks(B, orc, A, n, L, "dd", TOL, picks)
    wsp = check_chunks(B, orc, A, n, L, "split", 1e-3, picks)
    log(f"40x40 complex: 16 chunks of 2^12, worst rel err FP64 {w64:.2e}, FP32-product {wsp:.2e}")


def test_real48_chunk_length_invariance_and_drift(B, orc, inp):
    """One 2^22-term range at chunk lengths 2^8..2^16: the same sum up to drift."""
    n = 48
    A = inp.real_gaussian(n, 20190403)
    dA = dev_cm(A)
    start, count = 3 << 40, 1 << 22
    vals = {}
    for lc in (8, 12, 16):
        r = B.perm_partial(dA, start, count, log2_chunk=lc, drift_check=True)
        vals[lc] = val(r)
        log(f"  L=2^{lc}: drift {r.max_drift:.2e}")
        assert 0.0 <= r.max_drift < 1e-12
    assert rel(vals[8], vals[12]) < 1e-11 and rel(vals[16], vals[12]) < 1e-10
    # the whole range against the oracle's direct evaluation (4M terms, O(n^2) each)
    want = orc.chunk_partial(A, start, 1 << 16)
    got = B.perm_partial(dA, start, 1 << 16, log2_chunk=12)
    assert rel(val(got), val(want)) < TOL


@pytest.mark.parametrize("kind", ["real", "complex", "int01"])
def test_maximum_size_64(B, orc, inp, kind):
    """n = 64 (the largest size): ranges at the start, in the middle and at the
    very end of the 2^63-term Gray range, aligned and unaligned."""
    n = 64
    if kind == "real":
        A = inp.real_gaussian(n, 64)
    elif kind == "complex":
        A = inp.complex_gaussian(n, 64, scale=n ** -0.5)
    else:
        A = inp.bernoulli01(n, 64, p=0.1)
    dA = dev_cm(A)
    T = 1 << 63
    for start, count in ((0, 4096), (T - 4096, 4096), ((T // 3) | 5, 3000), (T - 777, 777)):
        got = B.perm_partial(dA, start, count)
        want = orc.chunk_partial(A, start, count)
        if kind == "int01":
            w = want - (1 << 128) if want >= (1 << 127) else want
            assert got.exact == w, (start, count)
        else:
            assert rel(val(got), val(want)) < TOL, (start, count)


def test_split_precision_reported_error(B, orc, inp):
    """FP32 products of FP64 row sums (row scaling on): the error is reported,
    not held to the FP64 bar; it grows with n (about 1e-6 at n = 16)."""
    for n in (12, 16, 20):
        A = inp.haar_block(n, n * n, 100 + n)
        want = val(orc.ryser(A))
        dd = rel(val(B.perm_complex(dev_cm(A))), want)
        sp = rel(val(B.perm_complex(dev_cm(A), precision="split")), want)
        log(f"  n={n}: FP64 {dd:.2e}  FP32-product {sp:.2e}")
        assert dd < TOL and sp < 1e-3


@pytest.mark.parametrize("n", [49, 56, 57, 63])
def test_large_complex_blocked_column_reads(B, orc, inp, n):
    """Complex n >= 49 reads each column in blocks of 8 rows (the last block
    shorter when 8 does not divide n): aligned chunks of 2^12 terms at the start,
    the end and inside the range against the oracle's direct terms, with the
    chunk-end drift check."""
    L = 1 << 12
    A = inp.complex_gaussian(n, 4900 + n, scale=n ** -0.5)
    picks = sampled_chunks(n, L, 6, n)
    worst = check_chunks(B, orc, A, n, L, "dd", TOL, picks)
    r = B.perm_partial(dev_cm(A), picks[2] * L, 64 * L, log2_chunk=12, drift_check=True)
    assert 0.0 <= r.max_drift < 1e-12
    log(f"  complex n={n}: 6 chunks of 2^12, worst rel err {worst:.2e}, drift {r.max_drift:.1e}")


@pytest.mark.parametrize("n", [49, 52, 55, 56, 60, 63, 64])
def test_large_complex_rows_in_lds(B, orc, inp, n):
    """From n = 49 the complex walk keeps rows 46.. of each lane's row sums in
    LDS (the drift-checked walk keeps them all in registers).  Checked against
    the oracle's direct terms in every precision, with one workgroup walking
    many chunks in turn (each lane's LDS rows re-formed at every chunk start),
    with chunks of 2 and 4 terms (the last pair alone, one pair before it),
    and over 2^26 terms against the all-register walk."""
    A = inp.complex_gaussian(n, 6400 + n, scale=n ** -0.5)
    dA = dev_cm(A)
    start = ((1 << (n - 1)) // 5) & ~((1 << 26) - 1)
    want = val(orc.chunk_partial(A, start, 1 << 14))
    for prec, tol in (("dd", TOL), ("fp64", TOL), ("split", 1e-3)):
        got = B.perm_partial(dA, start, 1 << 14, log2_chunk=4, blocks=1, precision=prec)
        assert rel(val(got), want) < tol, prec
    small = val(orc.chunk_partial(A, start, 1 << 10))
    for lc in (1, 2):
        got = B.perm_partial(dA, start, 1 << 10, log2_chunk=lc)
        assert rel(val(got), small) < TOL, lc
    a = val(B.perm_partial(dA, start, 1 << 26, log2_chunk=12))
    b = val(B.perm_partial(dA, start, 1 << 26, log2_chunk=12, drift_check=True))
    assert rel(a, b) < 1e-12
    log(f"  complex n={n} (rows in LDS): 2^14 terms in 1024 chunks on one workgroup, "
        f"2^26 terms vs the register walk {rel(a, b):.1e}")
