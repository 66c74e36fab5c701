"""Host logic of the sliced long-run driver, on the CPU.

``run_sliced`` only divides the Gray range and keeps the checkpoint; the
slice partials are added, with the factor 2(-1)^n of App. A (permanent), by
the library's host-only ``perm_combine``.  Here the GPU call is replaced,
inside the test only, by the oracle's partial sum over the same range, so the
slicing, resume and the C-ABI's final sum are checked against the oracle's
whole permanent without a GPU.
"""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture
def lr(monkeypatch, orc):
    from paper_1904_06229_amd import binding, longrun
    calls = []

    def fake_partial(A, start, count, **opts):
        a = A.numpy()
        r = orc.chunk_partial(a, start, count)
        calls.append((start, count))
        kw = dict(max_drift=0.0, terms=count, chunks=1, log2_chunk=0, blocks=1,
                  kernel_ms=1.0, total_ms=1.0)
        if isinstance(r, int):
            return binding.Result(0.0, 0.0, 0.0, 0.0, r, **kw)
        if hasattr(r, "re"):
            return binding.Result(r.re.hi, r.re.lo, r.im.hi, r.im.lo, None, **kw)
        return binding.Result(r.hi, r.lo, 0.0, 0.0, None, **kw)

    monkeypatch.setattr(binding, "perm_partial", fake_partial)
    longrun.calls = calls
    return longrun


def mats(n, seed):
    r = np.random.default_rng(seed)
    return {
        "real": r.standard_normal((n, n)),
        "complex": r.standard_normal((n, n)) + 1j * r.standard_normal((n, n)),
        "int01": (r.random((n, n)) < 0.5).astype(np.uint8),
    }


@pytest.mark.parametrize("n", [1, 2, 5, 9, 10])
@pytest.mark.parametrize("kind", ["real", "complex", "int01"])
def test_sliced_equals_whole(lr, orc, n, kind):
    A = mats(n, 40 + n)[kind]
    want = orc.ryser(A)
    T = 1 << (n - 1)
    for slices in sorted({1, min(2, T), min(4, T), T}):
        v, info = lr.run_sliced(torch.from_numpy(A), slices=slices)
        assert info["resumed"] == 0 and len(info["kernel_ms"]) == slices
        assert v.terms == T
        if kind == "int01":
            assert v.exact == want
        elif kind == "real":
            assert abs(v.value - float(want.exact)) <= 1e-12 * max(1.0, abs(float(want.exact)))
        else:
            w = complex(float(want.re.exact), float(want.im.exact))
            got = complex(v.re_hi + v.re_lo, v.im_hi + v.im_lo)
            assert abs(got - w) <= 1e-12 * max(1.0, abs(w))


def test_slices_cover_range_once(lr):
    A = mats(8, 7)["real"]
    lr.calls.clear()
    lr.run_sliced(torch.from_numpy(A), slices=8)
    assert lr.calls == [(k * 16, 16) for k in range(8)]


def test_resume_skips_done_slices_and_keeps_bits(lr, tmp_path):
    A = torch.from_numpy(mats(9, 3)["complex"])
    ck = tmp_path / "ck.jsonl"
    v1, _ = lr.run_sliced(A, slices=8, checkpoint=str(ck))
    lines = ck.read_text().splitlines()
    assert len(lines) == 8 and all(json.loads(x)["slices"] == 8 for x in lines)
    ck.write_text("\n".join(lines[:3]) + "\n")
    lr.calls.clear()
    v2, info = lr.run_sliced(A, slices=8, checkpoint=str(ck))
    assert info["resumed"] == 3 and [c[0] for c in lr.calls] == [k * 32 for k in range(3, 8)]
    bits = lambda r: (r.re_hi, r.re_lo, r.im_hi, r.im_lo)
    assert bits(v1) == bits(v2)  # fixed order of the final sum: same bits after resume


def test_checkpoint_of_other_matrix_ignored(lr, tmp_path):
    ck = tmp_path / "ck.jsonl"
    m = mats(7, 5)
    lr.run_sliced(torch.from_numpy(m["real"]), slices=4, checkpoint=str(ck))
    other = m["real"].copy()
    other[0, 0] += 1.0
    lr.calls.clear()
    _, info = lr.run_sliced(torch.from_numpy(other), slices=4, checkpoint=str(ck))
    assert info["resumed"] == 0 and len(lr.calls) == 4
    _, info = lr.run_sliced(torch.from_numpy(m["real"]), slices=2, checkpoint=str(ck))
    assert info["resumed"] == 0  # another slicing is not mixed in


@pytest.mark.parametrize("slices", [0, 3, 64])
def test_bad_slices(lr, slices):
    with pytest.raises(ValueError):
        lr.run_sliced(torch.from_numpy(mats(6, 1)["real"]), slices=slices)


def test_combine_rejects_incomplete_or_inconsistent_parts(orc):
    """perm_combine checks that the parts cover the 2^(n-1) terms once, and for
    0/1 input that the total is a multiple of 2^(n-1)."""
    from paper_1904_06229_amd import binding as B
    A = mats(6, 2)["int01"]
    kw = dict(max_drift=-1.0, chunks=1, log2_chunk=0, blocks=1, kernel_ms=0.0, total_ms=0.0)
    parts = [B.Result(0.0, 0.0, 0.0, 0.0, orc.chunk_partial(A, k * 8, 8), terms=8, **kw)
             for k in range(4)]
    assert B.perm_combine("int01", 6, parts).exact == orc.ryser(A)
    with pytest.raises(B.PermError):
        B.perm_combine("int01", 6, parts[:3])  # 24 of 32 terms
    bad = list(parts)
    bad[0] = B.Result(0.0, 0.0, 0.0, 0.0, parts[0].exact + 1, terms=8, **kw)
    with pytest.raises(B.PermError):
        B.perm_combine("int01", 6, bad)  # not a multiple of 2^5
    with pytest.raises(B.PermError):
        B.perm_combine("real", 6, parts + parts[:1])  # more than 2^(n-1) terms


def test_combine_sign_and_order():
    """2(-1)^n S, with the parts added as double-double pairs: parts that
    cancel to far below their own size keep their low words."""
    from paper_1904_06229_amd import binding as B
    kw = dict(max_drift=-1.0, chunks=1, log2_chunk=0, blocks=1, kernel_ms=0.0, total_ms=0.0)
    p = [B.Result(2.0 ** 40, 0.0, 0.0, 0.0, None, terms=2, **kw),
         B.Result(3.0, 2.0 ** -60, -1.0, 0.0, None, terms=1, **kw),
         B.Result(-(2.0 ** 40), 0.0, 0.5, 0.0, None, terms=1, **kw)]
    odd = B.perm_combine("complex", 3, p)  # n = 3: factor -2
    assert (odd.re_hi, odd.re_lo) == (-6.0, -(2.0 ** -59))
    assert (odd.im_hi, odd.im_lo) == (1.0, 0.0)
    even = B.perm_combine("real", 4, p + [B.Result(0.0, 0.0, 0.0, 0.0, None, terms=4, **kw)])
    assert (even.re_hi, even.re_lo) == (6.0, 2.0 ** -59) and even.terms == 8
