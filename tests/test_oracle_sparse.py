"""Pins of the sparse oracle (App. B: greedypartition, sparsepermanent).

Restricting Eq. ryser to column sets that meet every block drops only zero
terms (a set missing a block leaves that block's row with a zero sum), so
the value is per(A) exactly: pinned to the definition, Ryser's full sum, the
exact integer Ryser, and the Fibonacci numbers of tridiagonal ones matrices.
The enumeration itself is pinned by brute force: every set meeting every
block appears exactly once, consecutive sets of the Gray order differ in one
column, and the count is 2^|T| prod (2^|S_l| - 1).
"""
import math

import numpy as np
import pytest


def sparse_matrix(n, p, seed, kind="real", diag=True):
    r = np.random.default_rng(seed)
    M = r.random((n, n)) < p
    if diag:
        np.fill_diagonal(M, True)
    if kind == "int":
        return M.astype(np.uint8)
    A = r.standard_normal((n, n))
    if kind == "complex":
        A = A + 1j * r.standard_normal((n, n))
    return np.where(M, A, 0)


def close(a, b, tol):
    if isinstance(b, int):
        return a == b
    if hasattr(b, "re"):
        x, y = complex(a.re.exact, a.im.exact), complex(b.re.exact, b.im.exact)
    else:
        x, y = float(a.exact), float(b.exact)
    return abs(x - y) <= tol * max(abs(y), 1e-300)


@pytest.mark.parametrize("kind", ["real", "complex", "int"])
@pytest.mark.parametrize("n,p", [(1, 0.5), (4, 0.3), (8, 0.2), (9, 0.5), (10, 0.9), (12, 0.1),
                                 (14, 0.15)])
def test_sparse_equals_permanent(orc, kind, n, p):
    A = sparse_matrix(n, p, 31 * n + int(100 * p), kind)
    got, terms = orc.sparse(A)
    assert 1 <= terms <= 2 ** n
    assert close(got, orc.ryser(A), 1e-13)
    if n <= 9:
        assert close(got, orc.brute(A), 1e-13)


def test_fewer_sets_than_ryser(orc):
    A = sparse_matrix(20, 0.05, 7, "int")
    got, terms = orc.sparse(A)
    assert got == orc.ryser(A)
    assert terms < 2 ** 20 // 8


@pytest.mark.parametrize("n", [2, 5, 13, 24])
def test_tridiagonal_fibonacci(orc, n):
    from paper_1904_06229_amd import inputs
    fib = [0, 1]
    while len(fib) < n + 2:
        fib.append(fib[-1] + fib[-2])
    assert orc.sparse(inputs.tridiagonal_ones(n))[0] == fib[n + 1]


def test_zero_row(orc):
    A = sparse_matrix(6, 0.5, 1, "int")
    A[3, :] = 0
    assert orc.sparse(A) == (0, 0)


def partition_blocks(blk):
    blocks = {}
    for j, b in enumerate(blk):
        if b >= 0:
            blocks.setdefault(b, set()).add(j)
    return [blocks[b] for b in sorted(blocks)]


@pytest.mark.parametrize("seed", range(6))
def test_partition_is_greedy_and_disjoint(orc, seed):
    n = 16
    A = sparse_matrix(n, 0.12, 100 + seed)
    nbr = [set(np.nonzero(A[i])[0]) for i in range(n)]
    blocks = partition_blocks(orc.sparse_partition(A))
    # each block is the column set of a row, blocks pairwise disjoint
    for S in blocks:
        assert any(S == nb for nb in nbr)
    for a in range(len(blocks)):
        for b in range(a + 1, len(blocks)):
            assert not (blocks[a] & blocks[b])
    # replay of the greedy choice: least degree first, lowest index on ties
    alive, want = set(range(n)), []
    while alive:
        k = min(alive, key=lambda i: (len(nbr[i]), i))
        alive.discard(k)
        alive -= {l for l in alive if nbr[l] & nbr[k]}
        want.append(nbr[k])
    assert blocks == want


def test_enumeration_is_exactly_the_restricted_sets(orc):
    n = 11
    A = sparse_matrix(n, 0.18, 5)
    blocks = partition_blocks(orc.sparse_partition(A))
    T = n - sum(len(S) for S in blocks)
    count = 2 ** T * math.prod(2 ** len(S) - 1 for S in blocks)
    assert orc.sparse(A)[1] == count
    seq = [orc.sparse_set(A, g) for g in range(count)]
    assert len(set(seq)) == count
    want = {J for J in range(1 << n)
            if all(any((J >> j) & 1 for j in S) for S in blocks)}
    assert set(seq) == want
    for a, b in zip(seq, seq[1:]):
        assert bin(a ^ b).count("1") == 1


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_gray_ranges_add_up(orc, kind):
    n = 12
    A = sparse_matrix(n, 0.2, 9, kind)
    whole, terms = orc.sparse(A)
    cuts = [0, 1, 17, terms // 3, terms // 3 + 1, terms]
    tot = [orc.sparse_range(A, a, b - a) for a, b in zip(cuts, cuts[1:])]
    if kind == "complex":
        s = sum(complex(t.re.exact, t.im.exact) for t in tot)
        w = complex(whole.re.exact, whole.im.exact)
    else:
        s = sum(float(t.exact) for t in tot)
        w = float(whole.exact)
    assert abs((-1) ** n * s - w) <= 1e-13 * abs(w)


def test_exact_integers_identity_plus_bernoulli(orc):
    """The paper's sparse timing matrices: ones on the diagonal, other
    entries 1 with probability p (Sec. II.D)."""
    for n, p in ((16, 0.05), (20, 0.1), (22, 0.02)):
        A = sparse_matrix(n, p, n, "int")
        assert orc.sparse(A)[0] == orc.ryser(A)


def _wrap128(v):
    v %= 1 << 128
    return v - (1 << 128) if v >= 1 << 127 else v


def test_exact_integer_ranges(orc):
    """sparse_range_int: the 0/1 range sum modulo 2^128.  Ranges add up to the
    whole sum, (-1)^n per(A) from the exact integer Ryser; single terms equal
    (-1)^|J| prod_i (ones of row i in J) formed here with Python integers for
    the set J of that Gray index, also where the products pass 2^64 (where a
    long-double sum would round)."""
    n = 13
    A = sparse_matrix(n, 0.25, 21, "int")
    _, terms = orc.sparse(A)
    cuts = [0, 1, 5, terms // 2, terms // 2 + 3, terms]
    tot = sum(orc.sparse_range_int(A, a, b - a) for a, b in zip(cuts, cuts[1:]))
    assert _wrap128(tot) == _wrap128((-1) ** n * orc.ryser(A))
    for n, p, seed in ((13, 0.25, 21), (30, 0.5, 3), (40, 0.6, 4)):
        A = sparse_matrix(n, p, seed, "int")
        Af = A.astype(np.float64)
        blocks = partition_blocks(orc.sparse_partition(Af))
        T = 2 ** (n - sum(len(S) for S in blocks)) * math.prod(2 ** len(S) - 1 for S in blocks)
        r = np.random.default_rng(seed)
        for g in [0, 1, 2, T - 1] + [int(x) for x in r.integers(0, T, size=5)]:
            J = orc.sparse_set(Af, g)
            cols = [j for j in range(n) if (J >> j) & 1]
            prod = 1
            for i in range(n):
                prod *= int(sum(int(A[i, j]) for j in cols))
            want = _wrap128((-1) ** len(cols) * prod)
            assert orc.sparse_range_int(A, g, 1) == want, (n, g)
        if n > 13:
            assert prod > 1 << 64 or prod == 0
