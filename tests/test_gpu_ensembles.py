"""GPU: random-ensemble permanent studies (Secs. III-VI) through perm_batched.

Pinned by (a) the oracle on subsamples of every ensemble, (b) distributions
that follow from the definition at n = 1 and 2, (c) the exact moments
E X^2 = 1 (every ensemble: unit-variance independent entries) and, for
Ginibre matrices, E X^4 = n + 1 (Sec. III), within their sampling error.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
stats = pytest.importorskip("scipy.stats")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1904_06229_amd import ensembles
    return ensembles


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.mark.parametrize("kind", ["gaussian", "circular", "bernoulli", "haar"])
def test_batch_values_vs_oracle(E, orc, kind):
    from paper_1904_06229_amd import inputs
    for n in (3, 9, 14):
        M = inputs.ensemble_batch(kind, n, 300, 11 * n, a=2.0)
        per = E.permanents(M).cpu().numpy()
        scale = math.sqrt(math.factorial(n))
        for k in range(0, 300, 15):
            w = orc.ryser(M[k])
            want = complex(w.re.hi + w.re.lo, w.im.hi + w.im.lo) if hasattr(w, "re") else w.hi + w.lo
            assert abs(per[k] - want) <= 1e-10 * max(abs(want), 1e-6 * scale), (n, k)


def test_n1_gaussian_is_rayleigh(E):
    """n = 1: X = |a| with a complex Gaussian of variance 1, so F(x) = 1 - exp(-x^2)."""
    X = E.sample_x("gaussian", 1, 20000, 5).cpu().numpy()
    p = stats.kstest(X, lambda x: 1.0 - np.exp(-x * x)).pvalue
    log(f"n=1 Ginibre vs Rayleigh: p = {p:.3f}")
    assert p > 1e-4


def test_n2_circular_closed_form(E):
    """n = 2, unit-modulus entries: per = e^{i alpha} + e^{i beta} with alpha - beta
    uniform, X^2 = 1 + cos(phi), F(x) = 1 - arccos(x^2 - 1)/pi on [0, sqrt 2]."""
    X = E.sample_x("circular", 2, 20000, 6).cpu().numpy()
    assert X.max() <= math.sqrt(2) + 1e-12
    F = lambda x: 1.0 - np.arccos(np.clip(x * x - 1.0, -1.0, 1.0)) / np.pi
    p = stats.kstest(X, F).pvalue
    log(f"n=2 circular vs closed form: p = {p:.3f}")
    assert p > 1e-4


def test_n2_bernoulli_two_values(E):
    """n = 2, +-1 entries: per = ab + cd is 0 or +-2 with probability 1/2 each."""
    m = 20000
    X = E.sample_x("bernoulli", 2, m, 7).cpu().numpy()
    zero = np.isclose(X, 0.0, atol=1e-12)
    assert np.all(zero | np.isclose(X, math.sqrt(2.0), rtol=1e-14))
    assert abs(zero.mean() - 0.5) < 5 * math.sqrt(0.25 / m)


@pytest.mark.parametrize("kind", ["gaussian", "circular", "bernoulli"])
def test_second_moment_is_one(E, kind):
    n, m = 8, 50000
    X = E.sample_x(kind, n, m, 8)
    x2 = (X ** 2).double()
    mean, sd = float(x2.mean()), float(x2.std())
    log(f"{kind} n={n}: <X^2> = {mean:.4f} +- {sd / math.sqrt(m):.4f}")
    assert abs(mean - 1.0) < 5 * sd / math.sqrt(m)


@pytest.mark.parametrize("n", [2, 3, 5])
def test_gaussian_fourth_moment(E, n):
    m = 200000
    X = E.sample_x("gaussian", n, m, 9 + n)
    x4 = (X ** 4).double()
    mean, sd = float(x4.mean()), float(x4.std())
    log(f"Ginibre n={n}: <X^4> = {mean:.3f} (n+1 = {n + 1}) +- {sd / math.sqrt(m):.3f}")
    assert abs(mean - (n + 1)) < 5 * sd / math.sqrt(m)


def test_ks_separates_and_accepts(E):
    """Two Ginibre samples pass a KS test at 0.1%; sqrt(n) U for a whole Haar
    unitary (the family S(n, n)) is clearly not Gaussian at n = 6."""
    n, m = 6, 20000
    g1 = E.sample_x("gaussian", n, m, 100)
    g2 = E.sample_x("gaussian", n, m, 200)
    s = E.sample_x("haar", n, m, 300, a=1.0)
    d_same, d_diff = E.ks_2samp(g1, g2), E.ks_2samp(g1, s)
    log(f"KS n={n}: Ginibre/Ginibre {d_same:.4f}, Ginibre/S(n,n) {d_diff:.4f}, "
        f"D_0.05 {E.ks_critical(0.05, m, m):.4f}")
    assert d_same < E.ks_critical(0.001, m, m)
    assert d_diff > 3 * E.ks_critical(0.05, m, m)


def test_study_outputs(E):
    res = E.study("circular", [4, 6], 5000, 12)
    x = np.array(res["x"])
    for n in (4, 6):
        r = res["per_n"][n]
        F = np.array(r["F"])
        assert np.all(np.diff(F) >= 0) and F[0] >= 0 and F[-1] <= 1
        assert len(r["f"]) == len(x) - 2 and len(r["eps"]) == len(x)
        assert abs(r["moments"][1] - 1.0) < 0.2
