"""GPU parity of the repeated-column walk (Sec. II.A, Eq. ryser2) against the oracle.

Whole permanents are compared with the oracle's weighted Ryser sum (and with
the dense GPU path on the expanded matrix); partial sums over ranges of the
reflected mixed-radix Gray order with the oracle's range form, whose digits
come from the top-down definition of that order.  FP64 tolerance 1e-10
relative, as for the dense path.
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


def dev(C):
    return torch.from_numpy(np.asfortranarray(C)).to("cuda")


def val(x):
    if hasattr(x, "re_hi"):
        return complex(x.re_hi + x.re_lo, x.im_hi + x.im_lo)
    if hasattr(x, "re"):
        return complex(x.re.hi + x.re.lo, x.im.hi + x.im.lo)
    return complex(x.hi + x.lo, 0.0)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def columns(n_rows, mult, seed, cplx):
    r = np.random.default_rng(seed)
    C = r.standard_normal((n_rows, len(mult)))
    if cplx:
        C = (C + 1j * r.standard_normal((n_rows, len(mult)))) / math.sqrt(2 * n_rows)
    return C


def term_mass(C, mult):
    """sum_f prod_k C(m_k, f_k) prod_i |sum_k f_k c_ik|: the absolute size of
    the terms of Eq. ryser2, computed in chunks (sets the error scale)."""
    R = len(mult)
    radices = [m + 1 for m in mult]
    T = math.prod(radices)
    binom = [np.array([math.comb(m, f) for f in range(m + 1)], dtype=np.float64) for m in mult]
    total = 0.0
    for g0 in range(0, T, 1 << 16):
        g = np.arange(g0, min(T, g0 + (1 << 16)))
        f = np.empty((len(g), R), dtype=np.int64)
        q = g.copy()
        for k, r in enumerate(radices):
            f[:, k] = q % r
            q //= r
        W = np.ones(len(g))
        for k in range(R):
            W *= binom[k][f[:, k]]
        rows = f.astype(np.float64) @ C.T
        total += float(np.sum(W * np.prod(np.abs(rows), axis=1)))
    return total


def chunk_len(mult, b):
    return math.prod(m + 1 for m in mult[:b])


def assert_fp64(got, want, C, mult, b):
    """1e-10 relative, or -- where the terms of Eq. ryser2 cancel far below
    their own size (a column repeated many times acts like a block of J) --
    2 (n + L) units of FP64 rounding (2^-53) of the absolute term mass: n
    rounded factors per product, at most L walked row-sum updates per chunk."""
    n = sum(mult)
    err = abs(val(got) - val(want))
    tol = max(TOL * abs(val(want)), 2 * (n + chunk_len(mult, b)) * 2.0 ** -53 * term_mass(C, mult))
    assert err <= tol, (val(got), val(want), err, tol)


PATTERNS = [[1], [3], [1, 1], [2, 1], [1, 2, 1], [2, 2, 2], [4, 1, 3], [5, 5], [3, 3, 3, 3],
            [1] * 12, [2] * 8, [1, 3, 5, 2, 1, 4], [7, 1, 1, 1, 2, 3], [20], [2] * 10 + [1] * 4,
            [6, 6, 6]]


@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
@pytest.mark.parametrize("mult", PATTERNS, ids=lambda m: "m" + "-".join(map(str, m)))
def test_whole_vs_oracle(B, orc, mult, cplx):
    n = sum(mult)
    C = columns(n, mult, 100 + n + len(mult), cplx)
    got = B.perm_repeated(dev(C), mult)
    want = orc.ryser2(C, mult)
    assert_fp64(got, want, C, mult, got.log2_chunk)


@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
def test_whole_vs_dense_path_on_expanded_matrix(B, orc, cplx):
    for mult in ([2, 3, 1, 4, 2], [1] * 6 + [3] * 4, [2, 1] * 6):
        n = sum(mult)
        C = columns(n, mult, 7 * n, cplx)
        A = np.repeat(C, mult, axis=1)
        dense = B.perm_complex(dev(A)) if cplx else B.perm_real(dev(A))
        rep = B.perm_repeated(dev(C), mult)
        assert rel(val(rep), val(dense)) < TOL
        assert rel(val(rep), val(orc.ryser(A))) < TOL


def test_all_multiplicities_one_equals_dense(B):
    r = np.random.default_rng(9)
    for n in (3, 10, 17):
        A = r.standard_normal((n, n))
        assert rel(val(B.perm_repeated(dev(A), [1] * n)), val(B.perm_real(dev(A)))) < TOL


@pytest.mark.parametrize("n", [1, 5, 12, 20, 30])
def test_single_distinct_column(B, n):
    """per = n! prod_i c_i.  With c_i = +-1 the terms C(n, f) f^n are
    integers; while they stay below 2^53 (n <= 12) the sum is exact.  Beyond
    that Eq. ryser2 cancels like Ryser's formula on J_n: the error bound is a
    few ulps of the largest partial sums, sum_f C(n, f) f^n 2^-50."""
    r = np.random.default_rng(n)
    c = r.choice([-1.0, 1.0], size=(n, 1))
    want = math.factorial(n) * int(np.prod(c))
    got = B.perm_repeated(dev(c), [n])
    if n <= 12:
        assert got.re_hi + got.re_lo == want
    else:
        bound = sum(math.comb(n, f) * f ** n for f in range(n + 1)) * 2.0 ** -50
        assert abs((got.re_hi + got.re_lo) - want) <= bound


@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
@pytest.mark.parametrize("lc", [1, 2, 3, 5, 8, 14])
def test_partial_ranges_vs_oracle(B, orc, cplx, lc):
    """Aligned and ragged ranges at several chunk caps (chunk = the first b
    digits, L = their radix product, head and tail summed one term per lane)."""
    mult = [2, 1, 3, 2, 1, 4, 2]
    n = sum(mult)
    C = columns(n, mult, 31, cplx)
    T = math.prod(m + 1 for m in mult)  # 3*2*4*3*2*5*3 = 2160
    dC = dev(C)
    for start, count in ((0, T), (0, 1), (T - 1, 1), (5, 1000), (17, T - 40), (720, 1080),
                         (1500, 659)):
        got = B.perm_repeated_partial(dC, mult, start, count, log2_chunk=lc)
        want = orc.ryser2_range(C, mult, start, count)
        assert rel(val(got), val(want)) < TOL, (start, count, lc)
        assert got.terms == count


def test_partials_add_up(B, orc):
    mult = [3, 2, 2, 1, 3, 1]
    n = sum(mult)
    C = columns(n, mult, 5, True)
    dC = dev(C)
    T = math.prod(m + 1 for m in mult)
    cuts = [0, 7, 100, 101, 400, T]  # T = 4*3*3*2*4*2 = 576
    tot = sum(val(B.perm_repeated_partial(dC, mult, a, b - a)) for a, b in zip(cuts, cuts[1:]))
    whole = val(B.perm_repeated(dC, mult))
    assert rel((-1) ** n * tot, whole) < TOL


def test_chunk_cap_invariance_and_reproducible(B, orc):
    """Every chunk cap gives the oracle's value to the FP64 bar (the sums are
    grouped differently, so they agree to rounding, not bit for bit); one cap
    repeated gives the same bits."""
    mult = [2] * 9 + [1] * 3
    n = sum(mult)
    C = columns(n, mult, 77, True)
    dC = dev(C)
    want = orc.ryser2(C, mult)
    for lc in (2, 4, 8, 12, 14):
        got = B.perm_repeated(dC, mult, log2_chunk=lc)
        assert_fp64(got, want, C, mult, got.log2_chunk)
    a = B.perm_repeated(dC, mult, log2_chunk=8)
    b = B.perm_repeated(dC, mult, log2_chunk=8)
    assert (a.re_hi, a.re_lo, a.im_hi, a.im_lo) == (b.re_hi, b.re_lo, b.im_hi, b.im_lo)


def test_row_scaling_and_layout(B, orc):
    mult = [2, 3, 1, 2]
    n = sum(mult)
    C = columns(n, mult, 3, False) * np.logspace(-30, 30, n)[:, None]
    want = val(orc.ryser2(C, mult))
    assert rel(val(B.perm_repeated(dev(C), mult)), want) < TOL
    assert rel(val(B.perm_repeated(dev(C), mult, row_scaling=False)), want) < TOL
    # row-major input and a padded leading dimension give the same value
    t = torch.from_numpy(np.ascontiguousarray(C)).to("cuda")
    assert rel(val(B.perm_repeated(t, mult)), want) < TOL
    big = torch.zeros((4, n + 5), dtype=torch.float64, device="cuda").t()
    big[:n].copy_(torch.from_numpy(C))
    assert rel(val(B.perm_repeated(big[:n], mult)), want) < TOL


def test_boson_sampling_collision_workload_chunks(B, orc, inp):
    """48 photons in 24 output modes, two in each: the 48 x 48 matrix has 24
    distinct columns of multiplicity 2 (3^24 terms).  Sampled chunks (first,
    last, random) against the oracle's range form."""
    n, R = 48, 24
    U = inp.haar_block(n, n * n, 20190406)
    C = np.ascontiguousarray(U[:, :R])
    mult = [2] * R
    dC = dev(C)
    T = 3 ** R
    L = 3 ** 7  # log2_chunk 12 -> b = 7 inner digits
    r = np.random.default_rng(24)
    picks = [0, T // L - 1] + [int(x) for x in r.integers(1, T // L - 1, size=6)]
    for c in picks:
        got = B.perm_repeated_partial(dC, mult, c * L, L, log2_chunk=12)
        want = orc.ryser2_range(C, mult, c * L, L)
        assert rel(val(got), val(want)) < TOL, c


def test_errors(B):
    C = dev(np.ones((4, 2)))
    for mult in ([1, 2], [0, 4], [2, 3]):
        with pytest.raises(B.PermError):
            B.perm_repeated(C, mult)
    with pytest.raises(B.PermError):
        B.perm_repeated(C, [2, 2], precision="split")
    with pytest.raises(B.PermError):
        B.perm_repeated(C, [2, 2], drift_check=True)
    with pytest.raises(B.PermError):
        B.perm_repeated_partial(C, [2, 2], 5, 5)  # 9 terms
    with pytest.raises(B.PermError):
        B.perm_repeated(dev(np.full((2, 2), np.nan)), [1, 1])
    # 64 distinct columns: 2^64 terms, beyond the index range (the dense path covers it)
    with pytest.raises(B.PermError):
        B.perm_repeated(dev(np.ones((64, 64))), [1] * 64)


def mixed_mult(n, seed, lead):
    """Multiplicities summing to n: `lead` first, then 1..3 drawn from a seed."""
    r = np.random.default_rng(seed)
    mult = list(lead)
    while sum(mult) < n:
        mult.append(int(min(r.integers(1, 4), n - sum(mult))))
    return mult


@pytest.mark.parametrize("n", [49, 52, 56, 60, 64])
def test_large_complex_rows_in_lds(B, orc, n):
    """From n = 49 the complex walk of Eq. ryser2 keeps rows 46.. of each
    lane's row sums in LDS.  Ranges of the reflected mixed-radix Gray order
    against the oracle's range form: one workgroup walking many chunks in turn
    (the LDS rows re-formed at every chunk start), chunks of odd length (nine
    terms: the unpaired last term), and the default plan."""
    for lead, lc, blocks in (([1, 1, 1, 1], 4, 1), ([2, 2], 4, 1), ([3, 1], 0, 0)):
        mult = mixed_mult(n, 700 + n, lead)
        C = columns(n, mult, 800 + n, True)
        T = math.prod(m + 1 for m in mult)
        dC = dev(C)
        for start, count in ((0, 1 << 14), (T // 3, 3000), (T - (1 << 13), 1 << 13)):
            got = B.perm_repeated_partial(dC, mult, start, count, log2_chunk=lc, blocks=blocks)
            want = orc.ryser2_range(C, mult, start, count)
            assert rel(val(got), val(want)) < TOL, (lead, start, count)
    log(f"  complex n={n} (rows in LDS): Eq. ryser2 ranges match the oracle")
