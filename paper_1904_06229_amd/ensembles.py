"""Random-matrix permanent studies on the GPU (Secs. III-VI).

The paper samples X = |per(A)| / sqrt(n!) for many random n x n matrices of
one ensemble (Ginibre, circular, +-1 Bernoulli, scaled Haar blocks) and
studies its moments, its distribution function F(x, n) = Pr(X <= x) on a
grid of 16 points per decade with the difference-quotient density and the
error sqrt(F (1 - F) / m) (Sec. III), and two-sample Kolmogorov-Smirnov
distances between ensembles (Sec. VI).

Every permanent is computed by the library's batched kernel (perm_batched);
the statistics are a few reductions and a sort over the X values, done with
torch on the device where the results already are.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding as B
from . import inputs


def permanents(mats: np.ndarray, stream=None, **opts):
    """per of every matrix of a (count, n, n) array (one size), via perm_batched.

    Returns a complex128 device tensor of length count.
    """
    import torch
    count, n, n2 = mats.shape
    if n != n2:
        raise ValueError("square matrices expected")
    is_complex = np.iscomplexobj(mats)
    # column-major blocks back to back: matrix k's (i, j) at k*stride + j*n + i
    cm = np.ascontiguousarray(np.transpose(mats, (0, 2, 1)))
    flat = cm.astype(np.complex128 if is_complex else np.float64).ravel()
    if is_complex:
        flat = flat.view(np.float64)
    stride = (2 if is_complex else 1) * n * n
    dA = torch.from_numpy(flat).to("cuda")
    out = torch.zeros(4 * count, dtype=torch.float64, device="cuda")
    st = torch.zeros(count, dtype=torch.int32, device="cuda")
    B.perm_batched(dA, [n] * count, [k * stride for k in range(count)], is_complex, out, st,
                   stream=stream, **opts)
    torch.cuda.synchronize()
    if int((st != 0).sum().item()) != 0:
        raise B.PermError(int(st[st != 0][0].item()), "perm_batched")
    o = out.view(count, 4)
    return torch.complex(o[:, 0] + o[:, 1], o[:, 2] + o[:, 3])


def sample_x(kind: str, n: int, count: int, seed: int, a: float = 2.0, batch: int = 20000,
             qr=None, **opts):
    """X = |per(A)| / sqrt(n!) for `count` matrices of the ensemble (device tensor)."""
    import torch
    xs = []
    for k, lo in enumerate(range(0, count, batch)):
        m = inputs.ensemble_batch(kind, n, min(batch, count - lo), seed + 7919 * k, a=a, qr=qr)
        xs.append(permanents(m, **opts).abs())
    return torch.cat(xs) / math.sqrt(math.factorial(n))


def moments(X, kmax: int = 4):
    """Sample moments <X^k>, k = 1..kmax (Sec. III)."""
    return [float((X ** k).mean().item()) for k in range(1, kmax + 1)]


def grid(x_lo: float, x_hi: float, per_decade: int = 16) -> np.ndarray:
    """x values in geometric progression, `per_decade` per decade, on powers 10^(j/per_decade)."""
    j0 = math.floor(math.log10(x_lo) * per_decade)
    j1 = math.ceil(math.log10(x_hi) * per_decade)
    return 10.0 ** (np.arange(j0, j1 + 1) / per_decade)


def cdf(X, x: np.ndarray) -> np.ndarray:
    """Empirical F(x) = Pr(X <= x) at the grid points."""
    import torch
    xs, _ = torch.sort(X)
    g = torch.as_tensor(x, dtype=xs.dtype, device=xs.device)
    return (torch.searchsorted(xs, g, right=True).double() / xs.numel()).cpu().numpy()


def density(F: np.ndarray, x: np.ndarray) -> np.ndarray:
    """f(x_i) = (F(x_{i+1}) - F(x_{i-1})) / (x_{i+1} - x_{i-1}) at the interior points."""
    return (F[2:] - F[:-2]) / (x[2:] - x[:-2])


def cdf_error(F: np.ndarray, m: int) -> np.ndarray:
    """epsilon(x) = sqrt(F (1 - F)) / sqrt(m) (Sec. III)."""
    return np.sqrt(F * (1.0 - F)) / math.sqrt(m)


def ks_2samp(X, Y) -> float:
    """Two-sample Kolmogorov-Smirnov distance D = sup_x |F(x) - G(x)| (Sec. VI).

    The supremum is attained at a sample point; both empirical CDFs are
    evaluated (right-continuous) at every point of the merged sample.
    """
    import torch
    xs, _ = torch.sort(X.reshape(-1).double())
    ys, _ = torch.sort(Y.reshape(-1).double().to(xs.device))
    z = torch.cat([xs, ys])
    fx = torch.searchsorted(xs, z, right=True).double() / xs.numel()
    fy = torch.searchsorted(ys, z, right=True).double() / ys.numel()
    return float((fx - fy).abs().max().item())


def ks_critical(alpha: float, m1: int, m2: int) -> float:
    """Large-sample rejection threshold D_alpha = c(alpha) sqrt((m1 + m2) / (m1 m2)),
    c(alpha) = sqrt(-ln(alpha / 2) / 2) (the Kolmogorov limit law)."""
    return math.sqrt(-math.log(alpha / 2.0) / 2.0) * math.sqrt((m1 + m2) / (m1 * m2))


def study(kind: str, sizes, count: int, seed: int, x_lo: float = 1e-3, x_hi: float = 10.0,
          a: float = 2.0, **opts) -> dict:
    """Moments and F(x, n), f(x, n), epsilon(x) for each n (Secs. III-V)."""
    x = grid(x_lo, x_hi)
    res = {"kind": kind, "count": count, "x": x.tolist(), "per_n": {}}
    for n in sizes:
        X = sample_x(kind, n, count, seed + 104729 * n, a=a, **opts)
        F = cdf(X, x)
        res["per_n"][n] = {"moments": moments(X), "F": F.tolist(),
                           "f": density(F, x).tolist(), "eps": cdf_error(F, count).tolist()}
    return res
