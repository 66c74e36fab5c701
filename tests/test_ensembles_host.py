"""Host checks of the ensemble-study statistics and generators (CPU tensors).

The statistics functions are device-agnostic torch code; here they run on
CPU tensors and are checked against scipy's routines and the paper's own
printed threshold (Sec. VI: D_0.05 = 0.00607 for two samples of 10^5).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
stats = pytest.importorskip("scipy.stats")


@pytest.fixture(scope="module")
def E():
    import importlib
    # the statistics need no GPU; importing the module loads the library's
    # binding, which only needs the built .so
    return importlib.import_module("paper_1904_06229_amd.ensembles")


def test_ks_critical_matches_paper(E):
    assert round(E.ks_critical(0.05, 10 ** 5, 10 ** 5), 5) == 0.00607


@pytest.mark.parametrize("m1,m2", [(100, 100), (1000, 357), (5000, 5000)])
def test_ks_2samp_matches_scipy(E, m1, m2):
    r = np.random.default_rng(m1 + m2)
    x = r.exponential(size=m1)
    y = r.exponential(scale=1.1, size=m2)
    want = stats.ks_2samp(x, y).statistic
    assert abs(E.ks_2samp(torch.from_numpy(x), torch.from_numpy(y)) - want) < 1e-12


def test_ks_2samp_with_ties(E):
    x = torch.tensor([0.0, 0.0, 1.0, 2.0, 2.0])
    y = torch.tensor([0.0, 1.0, 1.0, 1.0])
    want = stats.ks_2samp(x.numpy(), y.numpy()).statistic
    assert abs(E.ks_2samp(x, y) - want) < 1e-12


def test_grid_sixteen_per_decade(E):
    x = E.grid(1e-3, 10.0)
    assert np.allclose(np.log10(x) * 16, np.round(np.log10(x) * 16))
    assert x[0] <= 1e-3 * (1 + 1e-12) and x[-1] >= 10.0 * (1 - 1e-12)
    assert np.allclose(x[16:] / x[:-16], 10.0)


def test_cdf_density_error_on_a_known_law(E):
    """Exponential(1) samples: the empirical F, its difference-quotient density
    and the error estimate behave as the definitions say."""
    m = 200000
    X = torch.from_numpy(np.random.default_rng(1).exponential(size=m))
    x = E.grid(0.05, 3.0)
    F = E.cdf(X, x)
    eps = E.cdf_error(F, m)
    assert np.all(np.abs(F - (1 - np.exp(-x))) < 5 * eps + 1e-12)
    f = E.density(F, x)
    assert np.allclose(f, np.exp(-x[1:-1]), rtol=0.1)
    assert np.all(np.diff(F) >= 0)


def test_moments(E):
    X = torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64)
    assert np.allclose(E.moments(X, 3), [2.0, 14.0 / 3.0, 12.0], rtol=1e-15)


@pytest.mark.parametrize("kind", ["gaussian", "circular", "bernoulli", "haar"])
def test_ensemble_entries_have_unit_variance(kind):
    from paper_1904_06229_amd import inputs
    M = inputs.ensemble_batch(kind, 6, 4000, 3, a=2.0)
    assert M.shape == (4000, 6, 6)
    v = np.mean(np.abs(M) ** 2)
    assert abs(v - 1.0) < 0.02
    assert abs(np.mean(M)) < 0.02
    if kind == "circular":
        assert np.allclose(np.abs(M), 1.0)
    if kind == "bernoulli":
        assert set(np.unique(M)) == {-1.0, 1.0} and not np.iscomplexobj(M)


def test_haar_blocks_are_blocks_of_unitaries():
    from paper_1904_06229_amd import inputs
    n, a = 4, 1.0  # m = n: the whole unitary, sqrt(m) U
    M = inputs.ensemble_batch("haar", n, 50, 9, a=a)
    for S in M:
        U = S / math.sqrt(n)
        assert np.allclose(U.conj().T @ U, np.eye(n), atol=1e-12)
