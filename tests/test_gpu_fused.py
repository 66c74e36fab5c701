"""GPU: the one-launch path of small real and complex permanents.

perm_real / perm_complex with default options take one launch for n <= 24:
every workgroup stages its own copy of the matrix, walks its chunks, and the
last workgroup to finish adds the partials in workgroup order.  Checked here
against the oracle's long-double Ryser sum (Sec. II.A, Eq. ryser) at the FP64
bar, against the three-launch path (forced by an explicit grid), for
bit-reproducibility (the finish order does not depend on which workgroup ends
last), and for its completion counter surviving an error call.
"""
import sys
import time
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


def dev(A):
    return torch.from_numpy(np.ascontiguousarray(A)).to("cuda")


def cval(x):
    if isinstance(x, Fraction):
        return (x, Fraction(0))
    if hasattr(x, "re_hi"):
        return (Fraction(x.re_hi) + Fraction(x.re_lo), Fraction(x.im_hi) + Fraction(x.im_lo))
    if hasattr(x, "re"):
        return (x.re.exact, x.im.exact)
    return (x.exact, Fraction(0))


def rel(got, want):
    g, w = cval(got), cval(want)
    num = (g[0] - w[0]) ** 2 + (g[1] - w[1]) ** 2
    return float(num / (w[0] ** 2 + w[1] ** 2)) ** 0.5


def bits(r):
    return (r.re_hi, r.re_lo, r.im_hi, r.im_lo)


@pytest.mark.parametrize("n", [2, 3, 4, 6, 9, 14, 18, 21, 24])
@pytest.mark.parametrize("kind", ["real", "complex"])
def test_one_launch_vs_oracle_and_three_launches(B, orc, inp, kind, n):
    if kind == "real":
        A, fn = inp.real_gaussian(n, 700 + n), B.perm_real
    else:
        A, fn = inp.complex_gaussian(n, 800 + n, scale=n ** -0.5), B.perm_complex
    one = fn(dev(A))
    three = fn(dev(A), blocks=64)  # an explicit grid takes the three-launch path
    want = orc.ryser(A)
    e1, e3 = rel(one, want), rel(three, want)
    print(f"  {kind} n={n}: one launch {e1:.2e} ({one.blocks} workgroups), three {e3:.2e}",
          file=sys.stderr, flush=True)
    assert e1 < TOL and e3 < TOL
    assert 0.0 < one.kernel_ms <= one.total_ms
    assert bits(fn(dev(A))) == bits(one)


def test_one_launch_precisions_and_scaling(B, orc, inp):
    n = 19
    A = inp.complex_gaussian(n, 919, scale=n ** -0.5)
    want = orc.ryser(A)
    assert rel(B.perm_complex(dev(A), precision="fp64"), want) < TOL
    assert rel(B.perm_complex(dev(A), precision="split"), want) < 1e-3
    # entries far from 1 in both directions: the row scales keep the walk in
    # range, and per(2^k A) = 2^(kn) per(A) holds to rounding (here 2^(+-760))
    R = inp.real_gaussian(n, 920)
    a = B.perm_real(dev(R * 2.0 ** 40))
    b = B.perm_real(dev(R * 2.0 ** -40))
    assert np.isfinite(a.re_hi) and b.re_hi != 0.0
    assert rel(b, (Fraction(a.re_hi) + Fraction(a.re_lo)) * Fraction(2) ** (-80 * n)) < 1e-13
    assert rel(a, orc.ryser(R * 2.0 ** 40)) < TOL
    # row scaling is exact: without it the same walk gives the same value here
    c = B.perm_real(dev(inp.real_gaussian(n, 921)))
    d = B.perm_real(dev(inp.real_gaussian(n, 921)), row_scaling=False)
    assert rel(c, d) < 1e-13


@pytest.mark.parametrize("kind,n", [("complex", 20), ("real", 13), ("complex", 9)])
def test_one_launch_chunk_lengths(B, orc, inp, kind, n):
    """Every chunk length takes the one launch, and with it the chunk starts
    whose part shared by a wave's lanes (all columns but b..b+6) comes from
    LDS: b = 1 puts the lanes' own columns at the bottom, larger b moves them
    up until none of the shared columns lie above them."""
    if kind == "real":
        A, fn = inp.real_gaussian(n, 1300 + n), B.perm_real
    else:
        A, fn = inp.complex_gaussian(n, 1400 + n, scale=n ** -0.5), B.perm_complex
    want = orc.ryser(A)
    three = fn(dev(A), blocks=64)
    for lc in range(1, min(8, n - 1) + 1):
        r = fn(dev(A), log2_chunk=lc)
        assert r.log2_chunk == lc and r.walk_variant == 1, (lc, r.walk_variant)
        assert rel(r, want) < TOL, lc
        assert rel(r, three) < 1e-13, lc


def test_one_launch_counter_survives_errors(B, inp):
    A = inp.complex_gaussian(16, 5, scale=0.25)
    before = B.perm_complex(dev(A))
    bad = A.copy()
    bad[7, 3] = complex(np.nan, 0.0)
    for _ in range(3):
        with pytest.raises(B.PermError) as e:
            B.perm_complex(dev(bad))
        assert e.value.status == B.PERM_ENONFINITE
    assert bits(B.perm_complex(dev(A))) == bits(before)


def test_one_launch_latency_reported(B, inp):
    """Median host time of 1000 20 x 20 complex calls (reported; the bar
    lives in the benchmark, not in a test)."""
    dA = dev(inp.complex_gaussian(20, 20190401, scale=20 ** -0.5))
    for _ in range(50):
        B.perm_complex(dA)
    ts = []
    for _ in range(1000):
        t0 = time.perf_counter()
        B.perm_complex(dA)
        ts.append(time.perf_counter() - t0)
    ts.sort()
    print(f"  20x20 complex: median {ts[500] * 1e6:.1f} us per call (python incl.)",
          file=sys.stderr, flush=True)
    assert ts[500] < 1e-3
