"""GPU parity of the sparse restricted Ryser walk (App. B) against the oracle.

Whole values against the oracle's own partition and sum (the value does not
depend on the partition), the device greedypartition against the oracle's
(integer work: identical), ranges of the Gray enumeration against the
oracle's range form, exact 0/1 results bit for bit (against the exact
integer oracle, and against the band oracle at n = 64 for band-shaped sparse
matrices), and the randomised trials.
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def dev(A):
    return torch.from_numpy(np.asfortranarray(A)).to("cuda")


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


def val(x):
    if hasattr(x, "re_hi"):
        return complex(x.re_hi + x.re_lo, x.im_hi + x.im_lo)
    if hasattr(x, "re"):
        return complex(x.re.hi + x.re.lo, x.im.hi + x.im.lo)
    return complex(x.hi + x.lo, 0.0)


def ryser_mass(A):
    """sum over all column sets J of prod_i |sum_{j in J} a_ij|: bounds the
    absolute size of the terms the restricted sum adds (n <= 18)."""
    n = A.shape[0]
    tot = 0.0
    for lo in range(0, 1 << n, 1 << 14):
        J = np.arange(lo, min(1 << n, lo + (1 << 14)))
        bits = ((J[:, None] >> np.arange(n)[None, :]) & 1).astype(np.float64)
        rows = bits @ A.T
        tot += float(np.sum(np.prod(np.abs(rows), axis=1)))
    return tot


def assert_fp64(got, want, A):
    err = abs(val(got) - val(want))
    n = A.shape[0]
    tol = max(TOL * abs(val(want)), 4 * n * 2.0 ** -53 * ryser_mass(A))
    assert err <= tol, (val(got), val(want), err, tol)


@pytest.mark.parametrize("kind", ["real", "complex"])
@pytest.mark.parametrize("n,p", [(1, 0.5), (5, 0.3), (9, 0.2), (12, 0.5), (14, 0.1), (16, 0.15),
                                 (18, 0.08)])
def test_whole_vs_oracle(B, orc, kind, n, p):
    A = sparse_matrix(n, p, 17 * n + int(100 * p), kind)
    got = B.perm_sparse(dev(A))
    want, terms = orc.sparse(A)
    assert got.terms == terms
    assert_fp64(got, want, A)


@pytest.mark.parametrize("n,p", [(8, 0.3), (16, 0.1), (24, 0.06), (30, 0.04), (34, 0.03)])
def test_int01_exact(B, orc, n, p):
    A = sparse_matrix(n, p, 5 * n, "int")
    got = B.perm_sparse(dev(A))
    want, terms = orc.sparse(A)
    log(f"0/1 sparse n={n} p={p}: per {want}, {terms} sets")
    assert got.exact == want and got.terms == terms


@pytest.mark.parametrize("n,p,seed", [(20, 0.4, 1), (24, 0.35, 2), (26, 0.5, 3), (28, 0.3, 4)])
def test_int01_exact_beyond_fp64_products(B, orc, n, p, seed):
    """Row degrees whose product is far above 2^53: the exact variant (integer
    bins) still gives the permanent bit for bit."""
    A = sparse_matrix(n, p, seed, "int")
    assert np.log2(A.sum(axis=1)).sum() > 60
    got = B.perm_sparse(dev(A))
    want = orc.ryser(A)
    log(f"0/1 n={n} p={p}: per {want}, {got.terms} sets, log2 prod deg "
        f"{np.log2(A.sum(axis=1)).sum():.0f}")
    assert got.exact == want


def test_int01_all_ones_and_range_guard(B):
    from paper_1904_06229_amd import inputs
    J = inputs.ones(30)  # one block of 30 columns is too large to restrict: 2^30 sets
    assert B.perm_sparse(dev(J)).exact == math.factorial(30)
    with pytest.raises(B.PermError) as e:
        B.perm_sparse(dev(inputs.ones(40)))  # Bregman: log2(40!) = 159 >= 127
    assert e.value.status == B.PERM_ERANGE


def test_int01_band_shaped_n64_against_band_oracle(B, orc):
    """n = 64: a sparse matrix inside a band of half-width 3 (zeros at random
    in the band, ones on the diagonal) has an exact value from the App. C
    transfer matrix, an independent algorithm."""
    n, k = 64, 3
    r = np.random.default_rng(64)
    i = np.arange(n)
    M = (np.abs(i[:, None] - i[None, :]) <= k) & (r.random((n, n)) < 0.08)
    np.fill_diagonal(M, True)
    A = M.astype(np.uint8)
    got = B.perm_sparse(dev(A), trials=16, seed=3)
    want = orc.band(A, k)
    log(f"band-shaped sparse n=64: per {want}, {got.terms} sets, kernel {got.kernel_ms:.1f} ms")
    assert got.exact == want


@pytest.mark.parametrize("n,p,seed,groups", [(40, 0.02, 1, 1), (40, 0.06, 2, 2), (40, 0.15, 3, 3),
                                             (48, 0.2, 4, 4), (48, 0.5, 5, 0)])
def test_int01_row_groups_exact(B, orc, n, p, seed, groups):
    """The exact walk deals the rows into the fewest equal groups (1..4) whose
    products of row degrees stay below 2^50, else falls back to groups of the
    size-only bound (0).  Each grouping against the oracle's exact integer
    range sums (mod 2^128), on ragged ranges at both ends and inside."""
    A = sparse_matrix(n, p, seed, "int")
    dA = dev(A)
    bits = float(np.log2(A.sum(axis=1)).sum())
    _, _, T = B.perm_sparse_partition(dA)
    count = (1 << 14) + 37
    r = np.random.default_rng(seed)
    for start in [0, T - count] + [int(x) for x in r.integers(0, T - count, size=3)]:
        got = B.perm_sparse_partial(dA, start, count)
        assert got.walk_variant == groups, (got.walk_variant, groups)
        assert groups == 0 or bits < 50 * groups
        want = orc.sparse_range_int(A, start, count)
        assert got.exact == want, (n, p, start)
    if T < 1 << 24:
        assert B.perm_sparse(dA).exact == orc.sparse(A)[0]
    log(f"0/1 n={n} p={p}: log2 prod deg {bits:.0f}, {groups} row groups, 2^{math.log2(T):.1f} sets")


@pytest.mark.parametrize("seed", range(5))
def test_partition_matches_oracle(B, orc, seed):
    for n, p in ((12, 0.2), (30, 0.06), (64, 0.02)):
        A = sparse_matrix(n, p, 1000 * seed + n)
        blk, nb, terms = B.perm_sparse_partition(dev(A))
        assert blk == orc.sparse_partition(A)
        assert nb == max(blk) + 1


def test_random_trials_never_worse(B, orc):
    A = sparse_matrix(40, 0.04, 77, "int")
    _, _, t1 = B.perm_sparse_partition(dev(A))
    _, _, t64 = B.perm_sparse_partition(dev(A), trials=64, seed=5)
    assert t64 <= t1
    a = B.perm_sparse(dev(A), trials=64, seed=5)
    b = B.perm_sparse(dev(A))
    assert a.exact == b.exact


@pytest.mark.parametrize("kind", ["real", "complex"])
@pytest.mark.parametrize("lc", [1, 3, 6, 10, 14])
def test_partial_ranges_vs_oracle(B, orc, kind, lc):
    n = 14
    A = sparse_matrix(n, 0.2, 3, kind)
    dA = dev(A)
    T = orc.sparse(A)[1]
    for start, count in ((0, T), (0, 1), (T - 1, 1), (7, T // 2), (T // 3, T - T // 3),
                         (T // 5, 333)):
        got = B.perm_sparse_partial(dA, start, count, log2_chunk=lc)
        want = orc.sparse_range(A, start, count)
        assert abs(val(got) - val(want)) <= max(TOL * abs(val(want)),
                                                 1e-13 * ryser_mass(A) / T * count), (start, count)


def test_int01_partial_sums_exact(B, orc):
    """Integer data: partial sums are integers below 2^53 here and must match exactly."""
    A = sparse_matrix(20, 0.08, 9, "int")
    T = orc.sparse(A)[1]
    for start, count in ((0, T), (3, T // 3), (T // 2, T - T // 2)):
        got = B.perm_sparse_partial(dev(A), start, count)
        want = orc.sparse_range(A, start, count)
        assert got.exact == int(want.exact), (start, count)
        assert got.re_hi + got.re_lo == float(want.exact), (start, count)


def test_paper_workload_chunks(B, orc):
    """The sparse timing matrices of Sec. II.D: ones on the diagonal, other
    entries 1 with probability p; n = 64, p = 0.01.  Sampled chunks of the
    Gray enumeration against the oracle's range form (exact integers)."""
    A = sparse_matrix(64, 0.01, 20190408, "int")
    blk, nb, T = B.perm_sparse_partition(dev(A))
    log(f"n=64 p=0.01: {nb} blocks, {T} sets (2^{math.log2(T):.1f})")
    r = np.random.default_rng(8)
    L = 1 << 10
    for s in [0, T - L] + [int(x) for x in r.integers(0, T - L, size=4)]:
        got = B.perm_sparse_partial(dev(A), s, L)
        want = orc.sparse_range(A, s, L)
        assert got.re_hi + got.re_lo == float(want.exact), s


def test_zero_row_and_errors(B):
    A = sparse_matrix(6, 0.5, 1, "int")
    A[2, :] = 0
    assert B.perm_sparse(dev(A)).exact == 0
    with pytest.raises(B.PermError):
        B.perm_sparse(dev(sparse_matrix(5, 0.5, 1)), trials=0)
    with pytest.raises(B.PermError):
        B.perm_sparse(dev(sparse_matrix(5, 0.5, 1)), precision="split")
    with pytest.raises(B.PermError):
        B.perm_sparse_partial(dev(sparse_matrix(5, 0.5, 1)), 0, 10 ** 6)
    bad = sparse_matrix(5, 0.5, 1)
    bad[1, 1] = np.inf
    with pytest.raises(B.PermError):
        B.perm_sparse(dev(bad))


def test_bench_workload_two_enumerations_exact(B, orc):
    """The benchmarked sparse workload at full size: n = 64, p = 0.02, seed
    20190408, App. B with 64 partition trials (seed 1).  Its exact permanent
    must equal, bit for bit, the one from the oracle's own partition (one
    greedy trial: another enumeration of other column sets), and sampled
    ranges of that enumeration match the oracle's exact integer sums."""
    A = sparse_matrix(64, 0.02, 20190408, "int")
    dA = dev(A)
    blk1, _, T1 = B.perm_sparse_partition(dA)
    blk64, _, T64 = B.perm_sparse_partition(dA, trials=64, seed=1)
    log(f"n=64 p=0.02: one trial {T1} sets (2^{math.log2(T1):.1f}), 64 trials {T64} sets "
        f"(2^{math.log2(T64):.1f}); partitions differ: {list(blk1) != list(blk64)}")
    assert T64 <= T1
    a = B.perm_sparse(dA, trials=64, seed=1)
    assert a.exact > 0
    if T1 <= 1 << 42:
        assert B.perm_sparse(dA).exact == a.exact
    for s, c in ((0, 1 << 16), (T1 - (1 << 12), 1 << 12), (T1 // 3, 4099)):
        got = B.perm_sparse_partial(dA, s, c)
        assert got.exact == orc.sparse_range_int(A, s, c), (s, c)
