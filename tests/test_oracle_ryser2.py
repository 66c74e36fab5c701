"""Pins of the repeated-column oracle (Sec. II.A, Eq. ryser2).

Eq. ryser2 is an identity: for the matrix A with column c_k repeated m_k
times it gives per(A) exactly.  The oracle's weighted sum over the vectors f
is pinned to routes that share none of its arithmetic: the n!-term
definition and the 2^n-subset Ryser sum of the expanded matrix, closed forms
(one distinct column: per = n! prod_i c_i), the plain Ryser sum when every
multiplicity is 1, and exact integers.  The mixed-radix Gray order of its
range form is pinned to the binary reflected code (all radices 2), to the
one-digit-per-step property and to covering every vector once.
"""
import math
from fractions import Fraction
from itertools import product

import numpy as np
import pytest


def expand(C, mult):
    return np.repeat(C, mult, axis=1)


def fr(x):
    if hasattr(x, "re"):
        return (x.re.exact, x.im.exact)
    return (x.exact, Fraction(0))


def close(a, b, tol):
    (ar, ai), (br, bi) = fr(a), fr(b)
    scale = max(abs(br), abs(bi), Fraction(1, 10 ** 30))
    return abs(ar - br) <= tol * scale and abs(ai - bi) <= tol * scale


PATTERNS = [[1], [2], [1, 1], [3, 1], [1, 2, 1], [2, 2, 2], [4, 1, 3], [1, 1, 1, 1, 1, 1, 1],
            [5, 5], [2, 3, 1, 2], [8], [1, 3, 5, 2, 1]]


@pytest.mark.parametrize("mult", PATTERNS, ids=lambda m: "m" + "-".join(map(str, m)))
@pytest.mark.parametrize("cplx", [False, True])
def test_equals_ryser_of_expanded_matrix(orc, mult, cplx):
    n, R = sum(mult), len(mult)
    r = np.random.default_rng(1000 + 7 * n + R)
    C = r.standard_normal((n, R))
    if cplx:
        C = C + 1j * r.standard_normal((n, R))
    A = expand(C, mult)
    assert close(orc.ryser2(C, mult), orc.ryser(A), 1e-15)
    if n <= 9:
        assert close(orc.ryser2(C, mult), orc.brute(A), 1e-15)


def test_all_multiplicities_one_is_plain_ryser(orc):
    r = np.random.default_rng(5)
    for n in (1, 4, 9, 13):
        A = r.standard_normal((n, n))
        assert close(orc.ryser2(A, [1] * n), orc.ryser(A), 1e-15)


@pytest.mark.parametrize("n", [1, 2, 5, 10, 17, 24])
def test_single_distinct_column_closed_form(orc, n):
    """All columns equal c: per = n! prod_i c_i (every permutation gives the same product)."""
    r = np.random.default_rng(n)
    c = r.integers(-3, 4, size=(n, 1)).astype(np.float64)
    c[c == 0] = 1.0
    want = math.factorial(n) * int(np.prod(c.astype(np.int64)))
    got = orc.ryser2(c, [n]).exact
    # The terms C(n, f) f^n prod c alternate in sign; each is formed with n
    # long-double roundings (2^-64), so the error is below n 2^-63 sum |term|.
    # Up to n = 12 every term and partial sum is an integer below 2^64: exact.
    bound = sum(math.comb(n, f) * f ** n for f in range(n + 1)) * abs(want) // math.factorial(n)
    if n <= 12:
        assert got == want
    else:
        assert abs(got - want) <= Fraction(n * bound, 2 ** 63)


def test_integer_matrices_exact(orc):
    """Small-integer distinct columns: the long-double sum is exact, equal to
    the exact integer brute force of the expanded 0/1 matrix."""
    r = np.random.default_rng(11)
    for mult in ([2, 1, 3], [1, 1, 2, 2], [3, 3, 2], [4, 4]):
        n = sum(mult)
        C = (r.random((n, len(mult))) < 0.6).astype(np.uint8)
        want = orc.brute(expand(C, mult))
        got = orc.ryser2(C.astype(np.float64), mult)
        assert got.exact == want


def test_row_repeats_by_transpose(orc):
    """Repeated rows: per(A) = per(A^T), so the rows are passed as columns."""
    r = np.random.default_rng(3)
    rows = r.standard_normal((3, 7))
    mult = [3, 2, 2]
    A = np.repeat(rows, mult, axis=0)
    assert close(orc.ryser2(rows.T, mult), orc.ryser(A), 1e-15)


def test_gray_order_binary_case(orc):
    """All radices 2: the order is the binary reflected Gray code g ^ (g >> 1)."""
    R = 10
    for g in range(1 << R):
        f = orc.mixed_gray(g, [2] * R)
        x = g ^ (g >> 1)
        assert f == [(x >> j) & 1 for j in range(R)]


@pytest.mark.parametrize("radices", [[3, 3], [2, 5, 3], [4, 2, 2, 3], [5], [3, 2, 4, 1, 2]])
def test_gray_order_visits_all_one_step_apart(orc, radices):
    T = math.prod(radices)
    seq = [tuple(orc.mixed_gray(g, radices)) for g in range(T)]
    assert seq[0] == tuple([0] * len(radices))
    assert sorted(seq) == sorted(product(*[range(r) for r in radices]))
    for a, b in zip(seq, seq[1:]):
        d = [abs(x - y) for x, y in zip(a, b)]
        assert sum(d) == 1


@pytest.mark.parametrize("cplx", [False, True])
def test_gray_ranges_add_up(orc, cplx):
    mult = [2, 1, 3, 2]
    n, R = sum(mult), len(mult)
    r = np.random.default_rng(21)
    C = r.standard_normal((n, R)) + (1j * r.standard_normal((n, R)) if cplx else 0)
    T = math.prod(m + 1 for m in mult)
    cuts = [0, 1, 17, 40, 41, T]
    parts = [fr(orc.ryser2_range(C, mult, a, b - a)) for a, b in zip(cuts, cuts[1:])]
    s = (sum(p[0] for p in parts), sum(p[1] for p in parts))
    sign = -1 if n % 2 else 1
    whole = fr(orc.ryser2(C, mult))
    scale = max(abs(whole[0]), abs(whole[1]))
    assert abs(sign * s[0] - whole[0]) <= 1e-15 * scale
    assert abs(sign * s[1] - whole[1]) <= 1e-15 * scale


def test_argument_errors(orc):
    C = np.ones((4, 2))
    for bad in ([1, 2], [0, 4], [5, -1], [2, 2, 0]):
        with pytest.raises(ValueError):
            orc.ryser2(C, bad)
    with pytest.raises(ValueError):
        orc.ryser2_range(C, [2, 2], 9, 1)  # only 9 vectors f
