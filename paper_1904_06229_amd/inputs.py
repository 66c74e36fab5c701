"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no permanent arithmetic: it only draws matrices.  It is
the one piece that both the GPU path (benchmarks, tests) and the CPU oracle's
tests use, so both sides see bit-identical inputs for a given seed.

Random numbers come from numpy's PCG64 generator (the paper names only the
Box-Muller method for its Gaussians, Sec. III; the generator is a free
choice, and these draws are as good).

Matrices are returned as numpy arrays in natural (row, column) indexing; the
callers lay them out column-major when they hand them to a library.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def complex_gaussian(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Ginibre entries (g1 + i g2)/sqrt(2), g1, g2 iid N(0,1) (Sec. III), times ``scale``.

    With scale = n**-0.5 the real and imaginary parts are iid N(0, 1/(2n)).
    """
    r = rng(seed)
    g = r.standard_normal((n, n, 2))
    return (g[..., 0] + 1j * g[..., 1]) * (scale / np.sqrt(2.0))


def real_gaussian(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """iid N(0, scale^2) real entries."""
    return rng(seed).standard_normal((n, n)) * scale


def bernoulli01(n: int, seed: int, p: float = 0.5) -> np.ndarray:
    """iid Bernoulli(p) 0/1 entries as uint8."""
    return (rng(seed).random((n, n)) < p).astype(np.uint8)


def haar_columns(m: int, n: int, r: np.random.Generator) -> np.ndarray:
    """First n columns of an m x m Haar-random unitary (Sec. VI).

    QR of a complex Gaussian matrix, then each column of Q multiplied by the
    phase r_jj/|r_jj| of R's diagonal (the Mezzadri recipe the paper uses).
    The first n columns of QR(G)'s Q only depend on the first n columns of G,
    so a thin QR of an m x n Gaussian gives them exactly.
    """
    g = r.standard_normal((m, n, 2))
    G = (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)
    Q, R = np.linalg.qr(G, mode="reduced")
    d = np.diagonal(R)
    ph = d / np.abs(d)
    return Q * ph[None, :]


def haar_block(n: int, m: int, seed: int) -> np.ndarray:
    """Top-left n x n block U_n of an m x m Haar unitary (unscaled; Sec. VI)."""
    return haar_columns(m, n, rng(seed))[:n, :]


def haar_unitary(n: int, seed: int) -> np.ndarray:
    """A full n x n Haar-random unitary."""
    return haar_columns(n, n, rng(seed))


def batched_haar_blocks(count: int, n_lo: int, n_hi: int, seed: int, qr=None):
    """``count`` matrices, n uniform on {n_lo..n_hi}, each the n x n top-left
    block of an n^2-mode Haar unitary (the paper's S(n^a, n) family at a = 2,
    unscaled, Sec. VI).

    Sizes are drawn first; then, size by size in increasing order, one
    Gaussian array for all matrices of that size and a stacked thin QR.
    Returns (list_of_sizes, list_of_matrices) in draw order.  ``qr`` may
    replace numpy's stacked QR (same contract: reduced Q and R of a stack).
    """
    qr = qr or (lambda G: np.linalg.qr(G, mode="reduced"))
    r = rng(seed)
    sizes = [int(x) for x in r.integers(n_lo, n_hi + 1, size=count)]
    mats = [None] * count
    by_n = {}
    for k, n in enumerate(sizes):
        by_n.setdefault(n, []).append(k)
    for n in sorted(by_n):
        idx = by_n[n]
        m = n * n
        for lo in range(0, len(idx), 2048):  # bounded memory per QR stack
            part = idx[lo:lo + 2048]
            g = r.standard_normal((len(part), m, n, 2))
            G = (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)
            Q, R = qr(G)
            d = np.diagonal(R, axis1=1, axis2=2)
            Q = Q * (d / np.abs(d))[:, None, :]
            for t, k in enumerate(part):
                mats[k] = np.ascontiguousarray(Q[t, :n, :])
    return sizes, mats


# ---- random-matrix ensembles (Secs. III-VI) ---------------------------------

ENSEMBLES = ("gaussian", "circular", "bernoulli", "haar")


def ensemble_batch(kind: str, n: int, count: int, seed: int, a: float = 2.0, qr=None):
    """``count`` n x n matrices of one ensemble, as a (count, n, n) array.

    gaussian  : Ginibre entries (g1 + i g2)/sqrt(2), mean 0, variance 1 (Sec. III)
    circular  : exp(i theta), theta uniform on [0, 2 pi) (Sec. IV)
    bernoulli : real +1 / -1 with probability 1/2 each (Sec. V)
    haar      : S = sqrt(m) U_n, U_n the top-left block of an m x m Haar
                unitary, m = round(n^a) (the family S(n^a, n) of Sec. VI)
    Every entry has variance 1, so E |per|^2 = n! in each ensemble
    (exactly for the first three).
    """
    r = rng(seed)
    if kind == "gaussian":
        g = r.standard_normal((count, n, n, 2))
        return (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)
    if kind == "circular":
        return np.exp(1j * r.uniform(0.0, 2.0 * np.pi, size=(count, n, n)))
    if kind == "bernoulli":
        return np.where(r.random((count, n, n)) < 0.5, 1.0, -1.0)
    if kind == "haar":
        qr = qr or (lambda G: np.linalg.qr(G, mode="reduced"))
        m = max(n, int(round(n ** a)))
        out = np.empty((count, n, n), dtype=np.complex128)
        for lo in range(0, count, 2048):
            k = min(2048, count - lo)
            g = r.standard_normal((k, m, n, 2))
            Q, R = qr((g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0))
            d = np.diagonal(R, axis1=1, axis2=2)
            out[lo:lo + k] = np.sqrt(m) * (Q * (d / np.abs(d))[:, None, :])[:, :n, :]
        return out
    raise ValueError(f"unknown ensemble {kind!r}; one of {ENSEMBLES}")


def band_batch(count: int, n: int, k: int, seed: int) -> np.ndarray:
    """``count`` complex n x n band matrices, a_ij = 0 for |i - j| > k, with
    Ginibre entries (g1 + i g2)/sqrt(2) on the band (App. C workloads), as a
    (count, n, n) array."""
    r = rng(seed)
    i = np.arange(n)
    mask = np.abs(i[:, None] - i[None, :]) <= k
    g = r.standard_normal((count, n, n)) + 1j * r.standard_normal((count, n, n))
    return np.where(mask, g, 0) / np.sqrt(2.0)


# ---- structured matrices with closed-form permanents -----------------------

def ones(n: int) -> np.ndarray:
    return np.ones((n, n), dtype=np.uint8)


def derangement_matrix(n: int) -> np.ndarray:
    """J - I: its permanent counts derangements."""
    return (np.ones((n, n)) - np.eye(n)).astype(np.uint8)


def menage_matrix(n: int) -> np.ndarray:
    """J - I - P (P the cyclic shift): its permanent is the menage number."""
    M = np.ones((n, n)) - np.eye(n) - np.roll(np.eye(n), 1, axis=1)
    return M.astype(np.uint8)


def tridiagonal_ones(n: int) -> np.ndarray:
    """1 where |i-j| <= 1: its permanent is the Fibonacci number F_{n+1}."""
    i = np.arange(n)
    return (np.abs(i[:, None] - i[None, :]) <= 1).astype(np.uint8)


def block_diag(*blocks) -> np.ndarray:
    dt = np.result_type(*blocks)
    n = sum(b.shape[0] for b in blocks)
    M = np.zeros((n, n), dtype=dt)
    o = 0
    for b in blocks:
        k = b.shape[0]
        M[o:o + k, o:o + k] = b
        o += k
    return M
