"""GPU: the partial sums behind a result (perm_opts.partials_out).

The library adds per-workgroup partial sums in a fixed order (the paper
stores partial sums in an array before its final compensated sum, Sec.
II.B).  With partials_out the caller gets that array: one record per
workgroup, scaled back to A itself.  Checked here: the records add up (as
exact rationals) to the call's own result -- App. A: per = 2 (-1)^n S for a
whole permanent, S itself for perm_partial -- and to the oracle's value;
0/1 records add up exactly modulo 2^128; the drift entries' maximum is the
call's max_drift; too small an array is refused; the entry points that do
not provide it say so.
"""
import sys
from fractions import Fraction

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1904_06229_amd import binding
    return binding


@pytest.fixture(scope="module")
def inp():
    from paper_1904_06229_amd import inputs
    return inputs


def dev_cm(A):
    return torch.from_numpy(np.asfortranarray(A)).to("cuda")


def fr(x):
    return Fraction(x)


def records(buf, parts):
    return buf[: 5 * parts].cpu().numpy().reshape(parts, 5)


def float_sum(rec):
    re = sum((fr(a) + fr(b) for a, b in rec[:, :2]), Fraction(0))
    im = sum((fr(a) + fr(b) for a, b in rec[:, 2:4]), Fraction(0))
    return re, im


def result_value(r):
    return fr(r.re_hi) + fr(r.re_lo), fr(r.im_hi) + fr(r.im_lo)


def rel(a, b):
    num = (a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2
    den = b[0] ** 2 + b[1] ** 2
    return float(num / den) ** 0.5


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_records_add_up_to_the_permanent(B, orc, inp, kind):
    n = 21
    A = inp.real_gaussian(n, 31) if kind == "real" else inp.complex_gaussian(n, 32, scale=n ** -0.5)
    fn = B.perm_real if kind == "real" else B.perm_complex
    buf = torch.full((5 * 6144,), np.nan, dtype=torch.float64, device="cuda")
    r = fn(dev_cm(A), partials=buf)
    assert 1 <= r.parts <= 6144 and r.walk_variant == 0  # the three-launch path
    rec = records(buf, r.parts)
    assert (rec[:, 4] == -1.0).all()
    s = float_sum(rec)
    sign = 2 if n % 2 == 0 else -2
    per = (sign * s[0], sign * s[1])
    assert rel(per, result_value(r)) < 1e-15
    w = orc.ryser(A)
    want = (w.re.exact, w.im.exact) if kind == "complex" else (w.exact, Fraction(0))
    assert rel(per, want) < 1e-10
    # the same bits as the call without records (which takes the one-launch path)
    assert rel(result_value(fn(dev_cm(A))), result_value(r)) < 1e-13
    print(f"  {kind} n={n}: {r.parts} records", file=sys.stderr, flush=True)


def test_partial_records_with_drift_and_row_scaling(B, orc, inp):
    n = 30
    A = inp.complex_gaussian(n, 33, scale=n ** -0.5) * 2.0 ** 20
    buf = torch.zeros(5 * 6144, dtype=torch.float64, device="cuda")
    start, count = 12345, (1 << 22) + 99
    r = B.perm_partial(dev_cm(A), start, count, drift_check=True, log2_chunk=10, partials=buf)
    rec = records(buf, r.parts)
    assert rel(float_sum(rec), result_value(r)) < 1e-15
    assert rec[:, 4].max() == r.max_drift and r.max_drift >= 0.0
    w = orc.chunk_partial(A, start, 1 << 14)
    got = B.perm_partial(dev_cm(A), start, 1 << 14, partials=buf)
    assert rel(float_sum(records(buf, got.parts)), (w.re.exact, w.im.exact)) < 1e-10
    # the no-allocation entry point fills the same records
    buf2 = torch.zeros_like(buf)
    r2 = B.perm_partial_noalloc(dev_cm(A), start, count, drift_check=True, log2_chunk=10,
                                partials=buf2)
    assert r2.parts == r.parts
    assert np.array_equal(records(buf2, r2.parts), rec)
    # the unaligned ends are single terms: their records carry drift 0
    assert (rec[:, 4] >= 0.0).all() and r2.max_drift == r.max_drift


def test_int01_records_add_up_exactly(B, orc, inp):
    n = 24
    A = inp.bernoulli01(n, 34)
    buf = torch.zeros(5 * 6144, dtype=torch.float64, device="cuda")
    r = B.perm_int01(dev_cm(A), partials=buf)
    rec = records(buf, r.parts).copy()
    words = rec[:, :2].view(np.uint64)
    total = 0
    for lo, hi in words:
        total = (total + (int(lo) | (int(hi) << 64))) % (1 << 128)
    if total >= 1 << 127:
        total -= 1 << 128
    # the records hold sum (-1)^(g+1) prod_i 2 w_i = (-1)^n 2^(n-1) per(A)
    assert total == (-1) ** n * 2 ** (n - 1) * orc.ryser(A)
    assert r.exact == orc.ryser(A)


def test_too_small_and_unsupported(B, inp):
    A = dev_cm(inp.real_gaussian(22, 35))
    small = torch.zeros(5 * 2, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PermError) as e:
        B.perm_real(A, partials=small, blocks=64)
    assert e.value.status == B.PERM_EINVAL
    C = torch.from_numpy(np.asfortranarray(inp.real_gaussian(6, 36)[:, :3])).to("cuda")
    with pytest.raises(B.PermError) as e:
        B.perm_repeated(C, [2, 2, 2], partials=small)
    assert e.value.status == B.PERM_ENOTIMPL
    # the library still works afterwards
    assert B.perm_real(A).terms == 1 << 21
