"""GPU: precision of the FP64 walks against the paper's own error fits (Sec. II.B).

per(J_n) = n! exactly, and J_n is the paper's precision test matrix: all
terms of the half-range sum have the same magnitude order and cancel
heavily.  The paper fits the relative error, in decimal digits, as
0.30 n - 17.2 for plain doubles summed over many cores and 0.20 n - 18 for
the double-quad (compensated) sum.  The FP64 walks here must stay within one
decade of those lines: the default double-double lane sum against the
double-quad fit, plain FP64 against the double fit.
"""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def B():
    from paper_1904_06229_amd import binding
    return binding


def rel_err_digits(r, n):
    got = Fraction(r.re_hi) + Fraction(r.re_lo)
    want = math.factorial(n)
    err = float(abs(got - want) / want)
    return math.log10(err) if err > 0 else -math.inf


@pytest.mark.parametrize("n", [12, 16, 20, 24, 28, 32, 36])
def test_ones_matrix_error_within_paper_fits(B, n):
    J = torch.ones((n, n), dtype=torch.float64, device="cuda")
    dd = rel_err_digits(B.perm_real(J), n)
    plain = rel_err_digits(B.perm_real(J, precision="fp64"), n)
    log(f"J_{n}: log10 rel err double-double {dd:.2f} (paper double-quad fit {0.20 * n - 18:.2f}), "
        f"plain FP64 {plain:.2f} (paper double fit {0.30 * n - 17.2:.2f})")
    assert dd <= 0.20 * n - 18 + 1
    assert plain <= 0.30 * n - 17.2 + 1
