"""GPU: a permanent as perm_partial slices (with checkpoint and resume)
equals the one-call permanent and the oracle."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def mods():
    from paper_1904_06229_amd import binding, inputs, longrun
    return binding, inputs, longrun


def dev_cm(A):
    return torch.from_numpy(np.asfortranarray(A)).to("cuda")


def test_sliced_real_and_complex(mods, orc):
    B, inp, lr = mods
    for n, A in ((24, inp.real_gaussian(24, 7)), (22, inp.haar_block(22, 484, 8))):
        dA = dev_cm(A)
        whole = B.perm_real(dA) if A.dtype == np.float64 else B.perm_complex(dA)
        v, info = lr.run_sliced(dA, slices=16)
        log(f"n={n}: 16 slices, {sum(info['seconds']):.3f} s")
        w = orc.ryser(A)
        if A.dtype == np.float64:
            got, want, one = v.re_hi + v.re_lo, float(w.exact), whole.re_hi + whole.re_lo
        else:
            got = complex(v.re_hi + v.re_lo, v.im_hi + v.im_lo)
            want = complex(float(w.re.exact), float(w.im.exact))
            one = complex(whole.re_hi + whole.re_lo, whole.im_hi + whole.im_lo)
        assert abs(got - want) <= 1e-10 * abs(want)
        assert abs(got - one) <= 1e-12 * abs(want)


def test_sliced_int01_exact_and_resume(mods, orc, tmp_path):
    B, inp, lr = mods
    n = 26
    A = inp.bernoulli01(n, 11)
    dA = dev_cm(A)
    want = orc.ryser(A)
    ck = tmp_path / "ck.jsonl"
    v, _ = lr.run_sliced(dA, slices=32, checkpoint=str(ck))
    assert v.exact == want == B.perm_int01(dA).exact
    lines = ck.read_text().splitlines()
    ck.write_text("\n".join(lines[:20]) + "\n")
    v2, info = lr.run_sliced(dA, slices=32, checkpoint=str(ck))
    assert info["resumed"] == 20 and v2.exact == v.exact


def test_sliced_real_resume_same_bits(mods, tmp_path):
    B, inp, lr = mods
    A = inp.real_gaussian(30, 9)
    dA = dev_cm(A)
    ck = tmp_path / "ck.jsonl"
    v1, _ = lr.run_sliced(dA, slices=8, checkpoint=str(ck))
    lines = ck.read_text().splitlines()
    ck.write_text("\n".join(lines[:5]) + "\n")
    v2, info = lr.run_sliced(dA, slices=8, checkpoint=str(ck))
    bits = lambda r: (r.re_hi, r.re_lo, r.im_hi, r.im_lo)
    assert info["resumed"] == 5 and bits(v1) == bits(v2)
    v3, _ = lr.run_sliced(dA, slices=8)  # fresh run: the walk is bit-reproducible
    assert bits(v3) == bits(v1)
