"""GPU parity of the batched path (one persistent launch over many matrices)."""
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


def pack(mats, is_complex):
    """Matrices back to back, each column-major with ld = n; offsets in doubles."""
    parts, offs, o = [], [], 0
    for M in mats:
        col = np.asfortranarray(M, dtype=np.complex128 if is_complex else np.float64)
        flat = col.ravel(order="F")
        if is_complex:
            flat = flat.view(np.float64)
        parts.append(flat)
        offs.append(o)
        o += flat.size
    return torch.from_numpy(np.concatenate(parts)).to("cuda"), offs


def run_batched(B, mats, is_complex, **kw):
    sizes = [M.shape[0] for M in mats]
    dA, offs = pack(mats, is_complex)
    out = torch.zeros(4 * len(mats), dtype=torch.float64, device="cuda")
    st = torch.full((len(mats),), -1, dtype=torch.int32, device="cuda")
    B.perm_batched(dA, sizes, offs, is_complex, out, st, **kw)
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(-1, 4)
    vals = [complex(r[0] + r[1], r[2] + r[3]) if is_complex else r[0] + r[1] for r in o]
    return vals, st.cpu().numpy(), (dA, sizes, offs, out, st)


def rel(a, b):
    return abs(a - b) / abs(b) if b != 0 else abs(a - b)


@pytest.mark.parametrize("is_complex", [True, False])
def test_mixed_sizes_vs_oracle(B, orc, inp, is_complex):
    r = np.random.default_rng(11)
    sizes = [1, 2, 3, 5, 8, 13, 17, 20, 24, 6, 9, 16, 21, 4, 12]
    sizes += [int(x) for x in r.integers(1, 25, size=25)]
    mats = []
    for k, n in enumerate(sizes):
        if is_complex:
            mats.append(inp.complex_gaussian(n, 500 + k, scale=n ** -0.5))
        else:
            mats.append(inp.real_gaussian(n, 500 + k))
    log(f"batched {'complex' if is_complex else 'real'}: {len(mats)} matrices")
    vals, st, _ = run_batched(B, mats, is_complex)
    assert (st == 0).all()
    for M, v in zip(mats, vals):
        w = orc.ryser(M)
        want = complex(w.re.hi + w.re.lo, w.im.hi + w.im.lo) if is_complex else w.hi + w.lo
        assert rel(v, want) < TOL, (M.shape[0], v, want)


def test_batched_matches_single(B, inp):
    """Same matrix (column-major A itself, not A^T), same chunks: the two paths
    walk identical chunks and differ only in reduction order.  Batched chunks
    of 2^8 terms; at n = 17..20 each lane walks two of their halves, so the
    single path takes 2^7-term chunks there.  The single calls take an explicit
    grid, hence the three-launch path, whose chunk starts are formed column by
    column in the batched walk's order (the one-launch path sums the columns
    shared by a wave first, a different rounding)."""
    mats = [inp.complex_gaussian(n, 900 + n, scale=n ** -0.5) for n in (10, 18, 22, 24, 32)]
    vals, st, _ = run_batched(B, mats, True, log2_chunk=8)
    for M, v in zip(mats, vals):
        col = torch.from_numpy(np.asfortranarray(M)).to("cuda")
        assert col.stride(0) == 1
        n = M.shape[0]
        s = B.perm_complex(col, log2_chunk=7 if 17 <= n <= 20 else 8, blocks=256).value
        assert rel(v, s) < 1e-15, n


def test_haar_blocks_unitary_bound(B, inp):
    sizes, mats = inp.batched_haar_blocks(200, 8, 16, seed=3)
    vals, st, _ = run_batched(B, mats, True)
    assert (st == 0).all()
    assert max(abs(v) for v in vals) <= 1.0


def test_nonfinite_flagged_per_matrix(B, inp):
    mats = [inp.real_gaussian(n, n) for n in (5, 7, 9)]
    mats[1][2, 3] = np.inf
    vals, st, _ = run_batched(B, mats, False)
    assert list(st) == [0, B.PERM_ENONFINITE, 0]
    assert math.isnan(vals[1]) and not math.isnan(vals[0]) and not math.isnan(vals[2])


def test_chunk_override_and_plain_fp64(B, orc, inp):
    mats = [inp.real_gaussian(n, 40 + n) for n in (11, 15, 19)]
    for kw in ({"log2_chunk": 1}, {"log2_chunk": 4}, {"precision": "fp64"}):
        vals, st, _ = run_batched(B, mats, False, **kw)
        for M, v in zip(mats, vals):
            w = orc.ryser(M)
            assert rel(v, w.hi + w.lo) < TOL


@pytest.mark.parametrize("lc", [0, 1, 2, 3, 9, 14])
def test_twin_chunk_sizes(B, orc, inp, lc):
    """Complex sizes 17..20 walk two half-length chunks of the same parity per
    lane in lockstep (tasks 2k and 2k + 1 together cover the chunks they cover
    one per lane).  Every chunk length against the oracle: 2 terms (b = 1:
    one chunk per lane), 4 terms (half-chunks of one pair), the default, and
    2^14 (fewer than 128 chunks per matrix: lanes past the end); n = 16 and 21
    walk one chunk per lane in the same launches."""
    mats = [inp.complex_gaussian(n, 300 + n, scale=n ** -0.5) for n in (16, 17, 18, 19, 20, 21)]
    mats += [inp.complex_gaussian(n, 400 + n, scale=n ** -0.5) for n in (17, 20)]
    vals, st, _ = run_batched(B, mats, True, log2_chunk=lc)
    assert (st == 0).all()
    for M, v in zip(mats, vals):
        w = orc.ryser(M)
        assert rel(v, complex(w.re.hi + w.re.lo, w.im.hi + w.im.lo)) < TOL, (M.shape[0], lc)


def test_graph_replay_matches_eager(B, inp):
    """Captured HIP graph: several replays, with eager work in between, each equal to eager."""
    mats = [inp.complex_gaussian(n, 70 + n, scale=n ** -0.5) for n in (6, 14, 19, 23)]
    eager, _, (dA, sizes, offs, out, st) = run_batched(B, mats, True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(4):
            out.zero_()
            B.perm_batched(dA, sizes, offs, True, out, st, stream=s, use_graph=True)
            s.synchronize()
            o = out.cpu().numpy().reshape(-1, 4)
            got = [complex(r[0] + r[1], r[2] + r[3]) for r in o]
            assert got == eager, f"replay {rep}"
            # unrelated eager work between replays
            B.perm_complex(torch.from_numpy(mats[0]).to("cuda"), stream=s)


def test_autotune_then_batched(B, orc, inp, tmp_path):
    path = str(tmp_path / "tune.json")
    B.perm_autotune(True, 8, 12, path)
    import json
    tab = json.load(open(path))
    assert set(tab["complex"]) == {str(n) for n in range(8, 13)}
    mats = [inp.complex_gaussian(n, 60 + n, scale=n ** -0.5) for n in range(8, 13)]
    vals, st, _ = run_batched(B, mats, True)
    for M, v in zip(mats, vals):
        w = orc.ryser(M)
        assert rel(v, complex(w.re.hi + w.re.lo, w.im.hi + w.im.lo)) < TOL


def test_argument_errors(B):
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    dA = torch.zeros(64 * 64, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PermError):
        B.perm_batched(dA, [33], [0], False, out)
    with pytest.raises(B.PermError):
        B.perm_batched(dA, [4], [0], False, out, precision="split")
    B.perm_batched(dA, [], [], False, out)  # empty batch is a no-op


def test_haar_batch_full_size_sampled(B, orc, inp):
    """The benchmarked batch at full size: 100000 complex Haar blocks, n uniform
    on 8..24 (seed 20190404), in the benchmark's launch configuration (HIP graph
    replay on a side stream).  Every status and value checked, an eager launch
    reproduces the graph's values bit for bit, and two matrices of every size
    against the oracle's Ryser sum."""
    def gpu_qr(G):  # stacked thin QR on the device (input generation only)
        Q, R = torch.linalg.qr(torch.from_numpy(G).to("cuda"), mode="reduced")
        return Q.cpu().numpy(), R.cpu().numpy()

    log("Haar batch: generating 100000 blocks, n 8..24, seed 20190404")
    sizes, mats = inp.batched_haar_blocks(100000, 8, 24, 20190404, qr=gpu_qr)
    dA, offs = pack(mats, True)
    count = len(sizes)
    out = torch.zeros(4 * count, dtype=torch.float64, device="cuda")
    st = torch.full((count,), -1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.perm_batched(dA, sizes, offs, True, out, st, stream=s, use_graph=True)
        B.perm_batched(dA, sizes, offs, True, out, st, stream=s, use_graph=True)
        s.synchronize()
    graph = out.cpu().numpy().reshape(-1, 4)
    assert (st.cpu().numpy() == 0).all() and np.isfinite(graph).all()
    out.zero_()
    B.perm_batched(dA, sizes, offs, True, out, st)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, 4), graph)
    log("Haar batch: values checked; oracle on two matrices of every size")
    first = {}
    r = np.random.default_rng(3)
    for k, n in enumerate(sizes):
        first.setdefault(n, []).append(k)
    for n in sorted(first):
        for k in (first[n][0], int(r.choice(first[n]))):
            w = orc.ryser(mats[k])
            want = complex(w.re.hi + w.re.lo, w.im.hi + w.im.lo)
            got = complex(graph[k][0] + graph[k][1], graph[k][2] + graph[k][3])
            assert rel(got, want) < TOL, (k, n, got, want)


def test_ginibre_ensemble_batch_full_size_sampled(B, orc, inp):
    """The benchmarked ensemble batch at full size: 100000 Ginibre 20 x 20
    matrices (seed 20190405), graph replay on a side stream.  Twenty sampled
    values against the oracle, and the sample mean of X^2 = |per|^2 / 20!
    against its exact expectation 1 (E|per|^2 = n! for iid unit-variance
    entries; Var X^2 = n for complex Gaussian entries, so the standard error
    of the mean is sqrt(20 / 100000) = 0.014)."""
    n, count = 20, 100000
    mats = inp.ensemble_batch("gaussian", n, count, 20190405)
    cm = np.ascontiguousarray(np.transpose(mats, (0, 2, 1))).astype(np.complex128)
    dA = torch.from_numpy(cm.ravel().view(np.float64)).to("cuda")
    sizes = np.full(count, n, dtype=np.int32)
    offs = np.arange(count, dtype=np.int64) * (2 * n * n)
    out = torch.zeros(4 * count, dtype=torch.float64, device="cuda")
    st = torch.full((count,), -1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.perm_batched(dA, sizes, offs, True, out, st, stream=s, use_graph=True)
        s.synchronize()
    o = out.cpu().numpy().reshape(-1, 4)
    assert (st.cpu().numpy() == 0).all() and np.isfinite(o).all()
    per = (o[:, 0] + o[:, 1]) + 1j * (o[:, 2] + o[:, 3])
    for k in np.random.default_rng(4).choice(count, 20, replace=False):
        w = orc.ryser(mats[k])
        assert rel(per[k], complex(w.re.hi + w.re.lo, w.im.hi + w.im.lo)) < TOL, k
    x2 = np.abs(per) ** 2 / math.factorial(n)
    log(f"Ginibre n=20: mean X^2 = {x2.mean():.4f} over {count}")
    assert abs(x2.mean() - 1.0) < 5 * math.sqrt(n / count)
