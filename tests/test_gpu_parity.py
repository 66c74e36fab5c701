"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Tolerances: floating-point results must agree with the oracle to a relative
error of 1e-10 (the FP64 bar; observed errors are far smaller at these
sizes); 0/1 results must be bit-exact.  Inputs are seeded draws from
``paper_1904_06229_amd.inputs``.
"""
import math
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


def dev(A):
    return torch.from_numpy(np.ascontiguousarray(A)).to("cuda")


def dev_cm(A):
    """Column-major device copy: the library sees A itself (a row-major tensor
    is read as A^T, which has the same permanent but other terms)."""
    t = torch.from_numpy(np.asfortranarray(A)).to("cuda")
    assert t.dim() < 2 or t.shape[0] < 2 or t.stride(0) == 1
    return t


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def frac_of(x):
    """(re, im) exact Fractions of an oracle value or a library Result."""
    if hasattr(x, "re_hi"):
        return (Fraction(x.re_hi) + Fraction(x.re_lo), Fraction(x.im_hi) + Fraction(x.im_lo))
    if hasattr(x, "exact") and not isinstance(x.exact, (int, type(None))):
        return (x.exact, Fraction(0))
    if hasattr(x, "re"):
        return (x.re.exact, x.im.exact)
    if isinstance(x, complex):
        return (Fraction(x.real), Fraction(x.imag))
    return (Fraction(x), Fraction(0))


def rel_err(got, want):
    gr, gi = frac_of(got)
    wr, wi = frac_of(want)
    num = math.sqrt(float((gr - wr) ** 2 + (gi - wi) ** 2))
    den = math.sqrt(float(wr ** 2 + wi ** 2))
    return num / den if den else num


# ------------------------------------------------------------ random ----

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 9, 12, 15, 16, 17, 20, 23, 24])
def test_real_gaussian(B, orc, inp, n):
    A = inp.real_gaussian(n, 1000 + n)
    log(f"real n={n}")
    got = B.perm_real(dev(A))
    want = orc.ryser(A)
    assert rel_err(got, want) < TOL
    if n <= 8:
        assert rel_err(got, orc.brute(A)) < TOL


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 8, 11, 13, 16, 19, 20, 22])
def test_complex_gaussian(B, orc, inp, n):
    A = inp.complex_gaussian(n, 2000 + n, scale=n ** -0.5)
    log(f"complex n={n}")
    got = B.perm_complex(dev(A))
    assert rel_err(got, orc.ryser(A)) < TOL


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 9, 13, 14, 16, 20, 22, 23, 24, 26])
def test_int01_bernoulli_exact(B, orc, inp, n):
    A = inp.bernoulli01(n, 3000 + n)
    log(f"int01 n={n}")
    got = B.perm_int01(dev(A))
    assert got.exact == orc.ryser(A)


def test_int01_config_30x30(B, orc, inp):
    """The 30x30 Bernoulli(1/2) workload, bit-exact against the integer Ryser oracle."""
    A = inp.bernoulli01(30, 20190413)
    log("int01 30x30 workload")
    got = B.perm_int01(dev(A))
    want = orc.ryser(A)
    log(f"  per = {want}, kernel {got.kernel_ms:.3f} ms, walk variant {got.walk_variant}")
    assert got.exact == want
    # sparsest column: 10 = n/3 ones; the next column flipped has 7 ones outside
    # those 10 rows (at most (n - n/3)/2 = 10): the banded walk
    assert got.walk_variant == 2


def with_sparse_column(rng, n, ones, p=0.5):
    """0/1 matrix with iid Bernoulli(p) entries, column 5 replaced by exactly `ones` ones."""
    A = (rng.random((n, n)) < p).astype(np.uint8)
    col = np.zeros(n, dtype=np.uint8)
    col[rng.choice(n, ones, replace=False)] = 1
    A[:, 5] = col
    return A


@pytest.mark.parametrize("n", [9, 12, 18, 21, 24, 26])
def test_int01_pair_shared_walk(B, orc, inp, n):
    """The pair-shared walk (sparsest column first; rows that column does not
    touch share one product per pair) engages exactly when that column has at
    most n/3 ones; both walks are exact."""
    rng = np.random.default_rng(7000 + n)
    M = n // 3
    for ones, engaged in ((M, True), (max(M - 2, 1), True), (M + 1, None)):
        A = with_sparse_column(rng, n, ones)
        want = orc.ryser(A)
        got = B.perm_int01(dev_cm(A))
        assert got.exact == want, (n, ones)
        plain = B.perm_int01(dev_cm(A), drift_check=True)  # drift check keeps the plain walk
        assert plain.exact == want and plain.walk_variant == 0
        if engaged:
            assert got.walk_variant in (1, 2), (n, ones)
        elif (A.sum(axis=0) > M).all():
            assert got.walk_variant == 0


@pytest.mark.parametrize("n", [9, 12, 18, 21, 24, 26])
def test_int01_banded_walk(B, orc, n):
    """The banded walk (column 1 flipped after every other pair; the rows with
    zeros in columns 0 and 1 share one product per two pairs) engages when a
    column has at most (n - n/3)/2 ones outside the first n/3 rows, and needs
    chunks of at least 4 terms; every walk is exact."""
    rng = np.random.default_rng(9000 + n)
    M = n // 3
    E = (n - M) // 2
    # band: column 5 has M ones, column 7 two ones (row sums below n keep every
    # group's product below 2^50 for n <= 30)
    A = with_sparse_column(rng, n, M)
    col = np.zeros(n, dtype=np.uint8)
    col[rng.choice(n, 2, replace=False)] = 1
    A[:, 7] = col
    want = orc.ryser(A)
    for lc, variant in ((0, 2), (2, 2), (3, 2), (1, 1)):
        got = B.perm_int01(dev_cm(A), log2_chunk=lc)
        assert got.exact == want, (n, lc)
        assert got.walk_variant == variant, (n, lc, got.walk_variant)
    # no band: every column but the sparse one is all ones, so more than E ones
    # outside the first M rows
    A2 = np.ones((n, n), dtype=np.uint8)
    col = np.zeros(n, dtype=np.uint8)
    col[rng.choice(n, M, replace=False)] = 1
    A2[:, 5] = col
    got = B.perm_int01(dev_cm(A2))
    assert got.exact == orc.ryser(A2) and got.walk_variant == 1, (n, got.walk_variant)
    assert n - M > E


def test_int01_banded_walk_block_diagonal_40(B, orc):
    """n = 40, beyond the oracle's whole 0/1 sums: a 20 (+) 20 block-diagonal
    Bernoulli(1/2) matrix, whose permanent is the product of its blocks',
    exactly, through the banded walk (2^39 terms)."""
    rng = np.random.default_rng(4040)
    n, h = 40, 20
    A = np.zeros((n, n), dtype=np.uint8)
    A[:h, :h] = rng.random((h, h)) < 0.5
    A[h:, h:] = rng.random((h, h)) < 0.5
    want = orc.ryser(A[:h, :h]) * orc.ryser(A[h:, h:])
    got = B.perm_int01(dev_cm(A))
    log(f"  40x40 block-diagonal 0/1: per = {want}, walk variant {got.walk_variant}, "
        f"walk {got.kernel_ms:.1f} ms")
    assert got.exact == want
    assert got.walk_variant == 2


def test_int01_pair_shared_not_for_dense(B, inp):
    r = B.perm_int01(dev(inp.ones(20)))
    assert r.walk_variant == 0 and r.exact == math.factorial(20)


# -------------------------------------------------------- structured ----

@pytest.mark.parametrize("n", [5, 13, 14, 22, 23, 27, 28])
def test_int01_ones_factorial(B, inp, n):
    assert B.perm_int01(dev(inp.ones(n))).exact == math.factorial(n)


def derangements(n):
    D = [1, 0]
    for k in range(2, n + 1):
        D.append((k - 1) * (D[-1] + D[-2]))
    return D[n]


@pytest.mark.parametrize("n", [2, 10, 21, 28])
def test_int01_derangements(B, inp, n):
    assert B.perm_int01(dev(inp.derangement_matrix(n))).exact == derangements(n)


def fib(k):
    a, b = 0, 1
    for _ in range(k):
        a, b = b, a + b
    return a


@pytest.mark.parametrize("n", [1, 2, 3, 12, 30, 34])
def test_int01_tridiagonal_fibonacci(B, inp, n):
    assert B.perm_int01(dev(inp.tridiagonal_ones(n))).exact == fib(n + 1)


@pytest.mark.parametrize("n", [10, 16, 20])
def test_fp64_tridiagonal_exact(B, inp, n):
    # every term is an integer below 2^53, so the double-double sum is exact
    r = B.perm_real(dev(inp.tridiagonal_ones(n).astype(np.float64)))
    assert r.re_hi + r.re_lo == fib(n + 1)


@pytest.mark.parametrize("n", [8, 12, 16, 20])
def test_fp64_ones_within_paper_error(B, n):
    """per(J_n) = n! (Sec. II.B); error within the paper's double-quad fit 10^(0.20n-18), one decade of margin."""
    r = B.perm_real(dev(np.ones((n, n))))
    err = rel_err(r, math.factorial(n))
    assert err < max(10 ** (0.20 * n - 18 + 1), 1e-15)


def test_block_diagonal_product(B, orc, inp):
    X = inp.real_gaussian(14, 41)
    Y = inp.real_gaussian(14, 42)
    M = inp.block_diag(X, Y)
    want = float(orc.ryser(X).exact * orc.ryser(Y).exact)
    assert rel_err(B.perm_real(dev(M)), want) < TOL


def test_unitary_bound(B, inp):
    U = inp.haar_block(24, 24 * 24, 5)
    r = B.perm_complex(dev(U))
    assert abs(r.value) <= 1.0


# ---------------------------------------------------------- partials ----

@pytest.mark.parametrize("kind", ["real", "complex", "int01"])
def test_partial_ranges_vs_chunk_oracle(B, orc, inp, kind):
    n = 18
    if kind == "real":
        A = inp.real_gaussian(n, 77)
    elif kind == "complex":
        A = inp.complex_gaussian(n, 78, scale=n ** -0.5)
    else:
        A = inp.bernoulli01(n, 79)
    T = 1 << (n - 1)
    r = np.random.default_rng(5)
    ranges = [(0, T), (0, 1), (T - 1, 1), (1, T - 1), (12345, 3), (4096, 8192)]
    for _ in range(6):
        s = int(r.integers(0, T))
        ranges.append((s, int(r.integers(0, T - s + 1))))
    for s, c in ranges:
        for lc in (0, 3, 7):
            got = B.perm_partial(dev(A), s, c, log2_chunk=lc)
            want = orc.chunk_partial(A, s, c)
            if kind == "int01":
                assert got.exact == (want - (1 << 128) if want >= (1 << 127) else want)
            elif c:
                assert rel_err(got, want) < TOL, (s, c, lc)
            else:
                assert got.value == 0


def test_partials_add_up_to_permanent(B, inp):
    """Splitting [0, 2^(n-1)) into pieces (how devices would share it) gives the permanent."""
    n = 20
    A = inp.complex_gaussian(n, 88, scale=n ** -0.5)
    T = 1 << (n - 1)
    whole = B.perm_complex(dev(A))
    cuts = [0, 1, 777, T // 3, T // 2 + 5, T]
    re = im = Fraction(0)
    for a, b in zip(cuts[:-1], cuts[1:]):
        p = B.perm_partial(dev(A), a, b - a)
        re += Fraction(p.re_hi) + Fraction(p.re_lo)
        im += Fraction(p.im_hi) + Fraction(p.im_lo)
    per = complex(float(2 * re), float(2 * im))  # n even: per = 2 S
    assert rel_err(whole, per) < 1e-12


# ------------------------------------------------------- invariances ----

def test_chunk_length_and_grid_invariance(B, orc, inp):
    """The sum does not depend on the split (Sec. II.B); only round-off does.

    Row sums are re-formed at every chunk start, so short chunks agree to a
    few ulps; longer walks add drift (about 5e-13 at 2^16 terms, n = 22)."""
    n = 22
    A = inp.real_gaussian(n, 99)
    want = orc.ryser(A)
    base = B.perm_real(dev(A))
    for lc in (1, 2, 5, 9, 12, 16):
        for blocks in (0, 1, 7, 333):
            r = B.perm_real(dev(A), log2_chunk=lc, blocks=blocks)
            assert rel_err(r, want) < TOL
            if lc <= 12:
                assert rel_err(r, base) < 1e-13
    I = inp.bernoulli01(24, 5)
    ib = B.perm_int01(dev(I)).exact
    for lc in (1, 2, 6, 10):
        for blocks in (0, 3, 100):
            assert B.perm_int01(dev(I), log2_chunk=lc, blocks=blocks).exact == ib


def test_bitwise_reproducible(B, inp):
    A = dev(inp.complex_gaussian(21, 5, scale=21 ** -0.5))
    r1 = B.perm_complex(A)
    r2 = B.perm_complex(A)
    assert (r1.re_hi, r1.re_lo, r1.im_hi, r1.im_lo) == (r2.re_hi, r2.re_lo, r2.im_hi, r2.im_lo)


def test_layouts_and_leading_dimension(B, inp):
    A = inp.complex_gaussian(17, 6, scale=17 ** -0.5)
    base = B.perm_complex(dev(A))
    T = dev(A).t()  # column-major view (stride(0) == 1)
    assert rel_err(B.perm_complex(T), base) < 1e-13
    big = np.zeros((20, 23), dtype=np.complex128)
    big[:17, :17] = A
    sub = dev(big)[:17, :17]  # ld = 23
    assert rel_err(B.perm_complex(sub), base) < 1e-13


def test_permutation_invariance(B, inp):
    A = inp.real_gaussian(19, 7)
    r = np.random.default_rng(0)
    base = B.perm_real(dev(A))
    P = A[r.permutation(19)][:, r.permutation(19)]
    assert rel_err(B.perm_real(dev(P)), base) < 1e-12


def test_row_scaling_exact_and_optional(B, inp):
    A = inp.real_gaussian(16, 8) * 1e-3
    a = B.perm_real(dev(A))
    b = B.perm_real(dev(A), row_scaling=False)
    assert rel_err(a, b) < 1e-13
    c = B.perm_real(dev(A * 2.0**-40))
    assert rel_err(c, (a.re_hi + a.re_lo) * 2.0 ** (-40 * 16)) < 1e-13


# ------------------------------------------------------ precisions ----

def test_precision_modes(B, orc, inp):
    n = 20
    A = inp.complex_gaussian(n, 2020, scale=n ** -0.5)
    want = orc.ryser(A)
    dd = rel_err(B.perm_complex(dev(A), precision="dd"), want)
    f64 = rel_err(B.perm_complex(dev(A), precision="fp64"), want)
    sp = rel_err(B.perm_complex(dev(A), precision="split"), want)
    log(f"n=20 complex rel err: dd {dd:.2e} fp64 {f64:.2e} split {sp:.2e}")
    assert dd < TOL and f64 < TOL
    assert sp < 1e-3  # FP32 products: reported, not held to the FP64 bar


def test_drift_check(B, inp):
    A = inp.real_gaussian(20, 3)
    r = B.perm_real(dev(A), drift_check=True, log2_chunk=12)
    assert 0.0 <= r.max_drift < 1e-12
    assert B.perm_real(dev(A)).max_drift == -1.0
    I = B.perm_int01(dev(inp.bernoulli01(20, 3)), drift_check=True)
    assert I.max_drift == 0.0


# ---------------------------------------------------------- errors ----

def test_edge_sizes(B):
    z = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    assert B.perm_real(z).value == 1.0
    a = torch.tensor([[-2.5]], dtype=torch.float64, device="cuda")
    assert B.perm_real(a).value == -2.5
    c = torch.tensor([[1.5 - 2j]], dtype=torch.complex128, device="cuda")
    assert B.perm_complex(c).value == 1.5 - 2j
    o = torch.tensor([[1]], dtype=torch.uint8, device="cuda")
    assert B.perm_int01(o).exact == 1


def test_error_paths(B, inp):
    A = inp.real_gaussian(10, 1)
    A[3, 4] = np.nan
    with pytest.raises(B.PermError) as e:
        B.perm_real(dev(A))
    assert e.value.status == B.PERM_ENONFINITE
    C = inp.complex_gaussian(9, 1)
    C[0, 0] = complex(np.inf, 0)
    with pytest.raises(B.PermError) as e:
        B.perm_complex(dev(C))
    assert e.value.status == B.PERM_ENONFINITE
    I = inp.bernoulli01(12, 1)
    I[2, 2] = 2
    with pytest.raises(B.PermError) as e:
        B.perm_int01(dev(I))
    assert e.value.status == B.PERM_EINVAL
    with pytest.raises(B.PermError) as e:
        B.perm_int01(dev(inp.ones(30)))
    assert e.value.status == B.PERM_ERANGE
    with pytest.raises(B.PermError) as e:
        B.perm_real(dev(inp.real_gaussian(8, 2)), log2_chunk=30)
    assert e.value.status == B.PERM_EINVAL
    # the library recovers after errors
    assert B.perm_int01(dev(inp.ones(6))).exact == 720
