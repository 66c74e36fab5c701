"""GPU parity of the band transfer matrix (App. C) against the oracle.

The transfer matrix has no inclusion-exclusion: its only cancellation is that
of the entries' signs.  The FP64 bar is 1e-10 relative, or n 2^-50 times
per(|A|) (the sum of the absolute values of all products) where that is
larger.  All-ones tridiagonal matrices give integers (Fibonacci numbers) that
the kernel reproduces bit for bit while they fit in 53 bits.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1904_06229_amd import binding
    return binding


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def band_matrix(n, k, seed, cplx, ones=False):
    r = np.random.default_rng(seed)
    i = np.arange(n)
    mask = np.abs(i[:, None] - i[None, :]) <= k
    if ones:
        return mask.astype(np.float64)
    A = r.standard_normal((n, n))
    if cplx:
        A = A + 1j * r.standard_normal((n, n))
    return np.where(mask, A, 0)


def run(B, mats, k, cplx, **kw):
    parts, offs, o = [], [], 0
    for M in mats:
        flat = np.asfortranarray(M, dtype=np.complex128 if cplx else np.float64).ravel(order="F")
        if cplx:
            flat = flat.view(np.float64)
        parts.append(flat)
        offs.append(o)
        o += flat.size
    dA = torch.from_numpy(np.concatenate(parts)).to("cuda")
    out = torch.full((4 * len(mats),), np.nan, dtype=torch.float64, device="cuda")
    st = torch.full((len(mats),), -1, dtype=torch.int32, device="cuda")
    B.perm_band(dA, [M.shape[0] for M in mats], offs, k, cplx, out, st, **kw)
    r = out.view(-1, 4).cpu().numpy()
    return [complex(x[0] + x[1], x[2] + x[3]) for x in r], st.cpu().numpy(), r


def want_and_tol(orc, A, k):
    w = orc.band(A, k)
    if hasattr(w, "re"):
        want = complex(float(w.re.exact), float(w.im.exact))
    else:
        want = complex(float(w.exact), 0.0)
    mass = float(orc.band(np.abs(A), k).exact)
    n = A.shape[0]
    return want, max(1e-10 * abs(want), n * 2.0 ** -50 * mass)


@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
def test_band_vs_oracle(B, orc, k, cplx):
    mats = [band_matrix(n, k, 100 * k + n, cplx) for n in (1, 2, 3, 7, 12, 20, 33, 64, 65, 130)]
    vals, st, _ = run(B, mats, k, cplx)
    assert (st == 0).all()
    for M, v in zip(mats, vals):
        want, tol = want_and_tol(orc, M, k)
        assert abs(v - want) <= tol, (M.shape[0], v, want, tol)


def test_long_band_matrices(B, orc):
    """n = 1000 and 3000: far beyond the dense path, linear in n here.  The
    entries are scaled so that |per| stays inside the double range (about
    0.44 per row for k = 3, 0.52 for k = 2 with these Gaussian entries)."""
    mats = [band_matrix(1000, 3, 1, True) * 0.44, band_matrix(3000, 2, 2, True) * 0.52]
    k = 3
    vals, st, _ = run(B, mats, k, True)
    assert (st == 0).all()
    for M, v in zip(mats, vals):
        w = orc.band(M, k)
        want = complex(float(w.re.exact), float(w.im.exact))
        log(f"n={M.shape[0]}: per {want:.6e}, rel err {abs(v - want) / abs(want):.2e}")
        assert abs(v - want) <= 1e-10 * abs(want)


def test_tridiagonal_fibonacci_exact(B):
    fib = [0, 1]
    while len(fib) < 80:
        fib.append(fib[-1] + fib[-2])
    ns = [1, 2, 10, 30, 64, 76]
    vals, st, r = run(B, [band_matrix(n, 1, 0, False, ones=True) for n in ns], 1, False)
    for n, row in zip(ns, r):
        assert row[0] == float(fib[n + 1]) and row[1] == 0.0, n


def test_full_band_equals_dense(B, orc):
    """k >= n - 1: every entry is in the band; compare with Ryser and the dense GPU walk."""
    r = np.random.default_rng(4)
    mats = [r.standard_normal((n, n)) for n in (2, 4, 6)]
    vals, st, _ = run(B, mats, 5, False)
    for M, v in zip(mats, vals):
        w = float(orc.ryser(M).exact)
        assert abs(v.real - w) <= 1e-12 * abs(w)
    A = band_matrix(30, 3, 9, False)
    d = B.perm_real(torch.from_numpy(np.asfortranarray(A)).to("cuda"))
    v = run(B, [A], 3, False)[0][0].real
    assert abs(v - (d.re_hi + d.re_lo)) <= 1e-10 * abs(v)


def test_out_of_band_entries_not_read(B):
    A = band_matrix(12, 2, 3, False)
    junk = A + np.where(A == 0, 1e300, 0)
    assert run(B, [A], 2, False)[0] == run(B, [junk], 2, False)[0]


def test_nonfinite_status_and_neighbours_unaffected(B, orc):
    good = band_matrix(9, 2, 5, False)
    bad = good.copy()
    bad[4, 5] = np.nan
    vals, st, _ = run(B, [good, bad, good], 2, False)
    assert list(st) == [0, 3, 0]
    want, tol = want_and_tol(orc, good, 2)
    assert abs(vals[0] - want) <= tol and vals[0] == vals[2]


def test_grid_invariance(B):
    mats = [band_matrix(n, 4, n, True) for n in range(1, 60, 3)]
    a = run(B, mats, 4, True)[2]
    b = run(B, mats, 4, True, blocks=3)[2]
    assert np.array_equal(a, b)


def test_errors(B):
    dA = torch.zeros(16, dtype=torch.float64, device="cuda")
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    for k in (-1, 6):
        with pytest.raises(B.PermError):
            B.perm_band(dA, [4], [0], k, False, out)
    with pytest.raises(B.PermError):
        B.perm_band(dA, [0], [0], 1, False, out)
    with pytest.raises(B.PermError):
        B.perm_band(dA, [4], [0], 1, False, out, log2_chunk=3)


def test_empty_and_single_matrix_batches(B, orc):
    """An empty batch is a no-op (the output is untouched); a batch of one
    matrix leaves three of the workgroup's four waves without work."""
    dA = torch.zeros(16, dtype=torch.float64, device="cuda")
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    B.perm_band(dA, [], [], 3, True, out)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 7.0).all()
    M = band_matrix(37, 4, 12, True)
    vals, st, _ = run(B, [M], 4, True)
    want, tol = want_and_tol(orc, M, 4)
    assert st[0] == 0 and abs(vals[0] - want) <= tol


def test_bench_sized_batch_sampled(B, orc):
    """The benchmarked workload at full size: 20000 complex 64 x 64 matrices,
    k = 5, in the default launch configuration (one wavefront per matrix, grid
    from the occupancy).  Sampled results against the oracle, every status and
    value checked, and a 7-workgroup launch (each wave then walks about 700
    matrices) reproduces every value bit for bit."""
    from paper_1904_06229_amd import inputs
    n, k, count, seed = 64, 5, 20000, 20190407
    mats = inputs.band_batch(count, n, k, seed)
    log(f"band batch: {count} x {n}x{n}, k = {k}, seed {seed}")
    vals, st, r = run(B, mats, k, True)
    assert (st == 0).all() and np.isfinite(r).all()
    picks = [0, 1, 2, 3, 4, 1023, 9999, 19996, 19997, 19998, 19999]
    picks += list(np.random.default_rng(7).choice(count, 13, replace=False))
    for m in picks:
        want, tol = want_and_tol(orc, mats[m], k)
        assert abs(vals[m] - want) <= tol, (m, vals[m], want, tol)
    r7 = run(B, mats, k, True, blocks=7)[2]
    assert np.array_equal(r, r7)
