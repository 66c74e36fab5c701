"""GPU: input edge cases of the staging kernels and overlapping calls.

* Rows whose entries lie near the ends of the double range: the power-of-two
  row scaling (exact; per(DA) = prod_i d_i per(A)) must keep the walk finite
  when the permanent is finite.
* The exact 0/1 sparse path (App. B) assumes entries 0 and 1; any other byte
  is an error, not a silently inexact result.
* Overlapping calls from several host threads on several streams give, each,
  the same bits as the same call made alone.
"""
import sys
import threading
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def dev_cm(A):
    return torch.from_numpy(np.asfortranarray(A)).to("cuda")


def cval(x):
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
    return (r.re_hi, r.re_lo, r.im_hi, r.im_lo, r.exact)


def test_rows_near_the_double_range(B, orc):
    """per [[1e308, 1e308], [1e-308, 2e-308]] = 3 (to the rounding of the
    decimal inputs); larger sizes with one huge and one tiny row."""
    A = np.array([[1e308, 1e308], [1e-308, 2e-308]])
    for f in (B.perm_real,):
        got = f(dev_cm(A))
        assert np.isfinite(got.re_hi)
        assert rel(got, orc.ryser(A)) < TOL
        assert abs(got.value - 3.0) < 1e-12
    r = np.random.default_rng(5)
    for n in (5, 13, 24):
        M = r.standard_normal((n, n))
        M[0] *= 1e307
        M[n - 1] *= 1e-307
        got = B.perm_real(dev_cm(M))
        assert rel(got, orc.ryser(M)) < TOL, n
        C = M + 1j * r.standard_normal((n, n)) * np.abs(M).max(axis=1, keepdims=True)
        assert rel(B.perm_complex(dev_cm(C)), orc.ryser(C)) < TOL, n
        # partial sums (no final scale) and the repeated-column path stage the same way
        cnt = min(40, (1 << (n - 1)) - 3)
        assert rel(B.perm_partial(dev_cm(M), 3, cnt), orc.chunk_partial(M, 3, cnt)) < TOL, n
    # the repeated-column path stages its own copy: the same 2 x 2 matrix as
    # two distinct columns of multiplicity one
    got = B.perm_repeated(dev_cm(A), [1, 1])
    assert np.isfinite(got.re_hi)
    assert rel(got, orc.ryser(A)) < TOL


def test_sparse_int01_rejects_entries_other_than_0_1(B, orc):
    r = np.random.default_rng(8)
    S = (r.random((20, 20)) < 0.15).astype(np.uint8)
    np.fill_diagonal(S, 1)
    assert B.perm_sparse(dev_cm(S)).exact == orc.sparse(S)[0]
    T = S.copy()
    T[4, 4] = 2
    for call in (lambda: B.perm_sparse(dev_cm(T)),
                 lambda: B.perm_sparse_partial(dev_cm(T), 0, 64)):
        with pytest.raises(B.PermError) as e:
            call()
        assert e.value.status == B.PERM_EINVAL
    # the pattern alone is still fine, and the library recovers
    assert B.perm_sparse_partition(dev_cm(T))[1] == B.perm_sparse_partition(dev_cm(S))[1]
    assert B.perm_sparse(dev_cm(S)).exact == orc.sparse(S)[0]


def _run_threads(jobs):
    """Run every job in its own host thread, each on its own stream; return
    their results in order (re-raising the first error)."""
    out = [None] * len(jobs)
    errs = []
    start = threading.Barrier(len(jobs))

    def work(k, job):
        try:
            s = torch.cuda.Stream()
            start.wait()
            with torch.cuda.stream(s):
                out[k] = job(s)
            s.synchronize()
        except Exception as ex:  # noqa: BLE001 - collected and re-raised below
            errs.append(ex)

    th = [threading.Thread(target=work, args=(k, j)) for k, j in enumerate(jobs)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    if errs:
        raise errs[0]
    return out


def test_overlapping_single_matrix_calls(B, inp, orc):
    """Four threads, four streams, dense calls of different sizes and kinds,
    three rounds each: every result has the bits of the same call alone."""
    mats = [("complex", dev_cm(inp.complex_gaussian(22, 1, scale=22 ** -0.5))),
            ("real", dev_cm(inp.real_gaussian(25, 2))),
            ("int01", dev_cm(inp.bernoulli01(24, 3))),
            ("partial", dev_cm(inp.real_gaussian(30, 4)))]
    fns = {"complex": B.perm_complex, "real": B.perm_real, "int01": B.perm_int01,
           "partial": lambda A, stream=None: B.perm_partial(A, 12345, 1 << 22, stream=stream)}
    alone = [bits(fns[k](A)) for k, A in mats]
    for rnd in range(3):
        got = _run_threads([lambda s, k=k, A=A: fns[k](A, stream=s) for k, A in mats])
        assert [bits(g) for g in got] == alone, rnd
    log(f"  4 threads x 3 rounds: bit-identical to the calls made alone")


def test_overlapping_turn_taking_calls(B, orc):
    """Repeated-column, sparse and band calls from three threads (they take
    turns on the device): same bits as alone."""
    r = np.random.default_rng(12)
    C = r.standard_normal((12, 4)) + 1j * r.standard_normal((12, 4))
    S = (r.random((24, 24)) < 0.2).astype(np.uint8)
    np.fill_diagonal(S, 1)
    n, k = 30, 3
    i = np.arange(n)
    Bd = np.where(np.abs(i[:, None] - i[None, :]) <= k, r.standard_normal((n, n)), 0.0)
    flat = torch.from_numpy(np.asfortranarray(Bd).ravel(order="F")).to("cuda")
    dC, dS = dev_cm(C), dev_cm(S)

    def band(stream=None):
        out = torch.zeros(4 * 64, dtype=torch.float64, device="cuda")
        B.perm_band(flat, [n] * 64, [0] * 64, k, False, out, stream=stream)
        return tuple(out.cpu().numpy().tolist())

    jobs = [lambda s: bits(B.perm_repeated(dC, [3, 4, 2, 3], stream=s)),
            lambda s: bits(B.perm_sparse(dS, stream=s)),
            lambda s: band(stream=s)]
    alone = [j(None) for j in jobs]
    for rnd in range(3):
        assert _run_threads(jobs) == alone, rnd


def test_batched_on_two_streams(B, inp):
    """The same batch enqueued from two threads on two streams (one plan,
    reused in stream order), then again with graph replay."""
    r = np.random.default_rng(4)
    sizes = [int(x) for x in r.integers(8, 19, size=300)]
    parts, offs, o = [], [], 0
    for m, n in enumerate(sizes):
        M = inp.complex_gaussian(n, 500 + m, scale=n ** -0.5)
        flat = np.asfortranarray(M).ravel(order="F").view(np.float64)
        parts.append(flat)
        offs.append(o)
        o += flat.size
    dA = torch.from_numpy(np.concatenate(parts)).to("cuda")
    ref = torch.zeros(4 * len(sizes), dtype=torch.float64, device="cuda")
    B.perm_batched(dA, sizes, offs, True, ref)
    torch.cuda.synchronize()
    want = ref.cpu().numpy()
    for graph in (False, True):
        outs = [torch.zeros_like(ref) for _ in range(2)]
        torch.cuda.synchronize()  # the fills run on this thread's stream

        def job(k):
            def run(s):
                for _ in range(3):
                    B.perm_batched(dA, sizes, offs, True, outs[k], stream=s, use_graph=graph)
                return None
            return run
        # both threads write their own output buffer through the shared plan
        _run_threads([job(0), job(1)])
        torch.cuda.synchronize()
        for k in range(2):
            assert np.array_equal(outs[k].cpu().numpy(), want), (graph, k)
