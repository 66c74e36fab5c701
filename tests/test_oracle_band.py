"""Pins of the band transfer-matrix oracle (App. C, bandpermanent).

The transfer matrix reaches the permanent exactly, so it is pinned to the
definition (brute force) and Ryser's sum on random band matrices, to the
Fibonacci numbers for the tridiagonal all-ones matrix (every permutation
with |pi(i) - i| <= 1 is a product of disjoint adjacent transpositions), and
to a direct count of permutations with displacement <= 2 for k = 2.
"""
import math
from itertools import permutations

import numpy as np
import pytest


def band_matrix(n, k, seed, kind):
    r = np.random.default_rng(seed)
    i = np.arange(n)
    mask = np.abs(i[:, None] - i[None, :]) <= k
    if kind == "int":
        return ((r.random((n, n)) < 0.7) & mask).astype(np.uint8)
    A = r.standard_normal((n, n))
    if kind == "complex":
        A = A + 1j * r.standard_normal((n, n))
    return np.where(mask, A, 0)


def close(a, b, tol=1e-15):
    if isinstance(b, int):
        return a == b
    if hasattr(b, "re"):
        a_, b_ = complex(a.re.exact, a.im.exact), complex(b.re.exact, b.im.exact)
    else:
        a_, b_ = float(a.exact), float(b.exact)
    return abs(a_ - b_) <= tol * max(abs(b_), 1e-300)


@pytest.mark.parametrize("kind", ["real", "complex", "int"])
@pytest.mark.parametrize("n,k", [(1, 0), (2, 1), (5, 1), (7, 2), (9, 3), (10, 2), (8, 7), (9, 9)])
def test_band_vs_definition(orc, kind, n, k):
    A = band_matrix(n, k, 10 * n + k, kind)
    assert close(orc.band(A, k), orc.brute(A), 1e-14)


@pytest.mark.parametrize("kind", ["real", "complex", "int"])
@pytest.mark.parametrize("n,k", [(14, 1), (16, 3), (18, 5), (13, 9)])
def test_band_vs_ryser(orc, kind, n, k):
    A = band_matrix(n, k, 7 * n + k, kind)
    assert close(orc.band(A, k), orc.ryser(A), 1e-13)


def test_wider_band_same_value(orc):
    """A band-k matrix is also a band-k' matrix for k' > k."""
    A = band_matrix(20, 2, 5, "real")
    v = [float(orc.band(A, k).exact) for k in (2, 3, 6, 9)]
    assert all(abs(x - v[0]) <= 1e-14 * abs(v[0]) for x in v)


@pytest.mark.parametrize("n", [1, 2, 3, 10, 30, 64, 90])
def test_tridiagonal_fibonacci(orc, n):
    from paper_1904_06229_amd import inputs
    fib = [0, 1]
    while len(fib) < n + 2:
        fib.append(fib[-1] + fib[-2])
    assert orc.band(inputs.tridiagonal_ones(n), 1) == fib[n + 1]


def displacement_count(n, k):
    return sum(1 for p in permutations(range(n)) if all(abs(p[i] - i) <= k for i in range(n)))


def test_displacement_two_counts(orc):
    """k = 2 all-ones band: the number of permutations moving no point by more
    than 2, counted directly for n <= 9; these counts satisfy
    a(n) = 2a(n-1) + 2a(n-3) - a(n-5), which then gives a(64)."""
    i64 = np.arange(64)
    ones = lambda n: (np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]) <= 2).astype(np.uint8)
    a = [1] + [displacement_count(n, 2) for n in range(1, 10)]
    for n in range(1, 10):
        assert orc.band(ones(n), 2) == a[n]
    for n in range(5, 10):
        assert a[n] == 2 * a[n - 1] + 2 * a[n - 3] - a[n - 5]
    while len(a) <= 64:
        m = len(a)
        a.append(2 * a[m - 1] + 2 * a[m - 3] - a[m - 5])
    assert orc.band(ones(64), 2) == a[64]
    del i64


def test_diagonal(orc):
    d = np.random.default_rng(2).standard_normal(12)
    assert close(orc.band(np.diag(d), 0), type(orc.band(np.diag(d), 0))(float(np.prod(d))), 1e-15)


def test_out_of_band_entry_rejected(orc):
    A = band_matrix(6, 1, 1, "real")
    A[0, 5] = 1.0
    with pytest.raises(ValueError):
        orc.band(A, 1)
    with pytest.raises(ValueError):
        orc.band(band_matrix(6, 1, 1, "real"), 10)  # k above the supported maximum
