"""Small seeded matrices for tests: decaying, block-structured, scaled blocks.

Input generation only (no SpAMM or SP2 arithmetic); shared by the oracle
tests and the device parity tests.
"""
from __future__ import annotations

import numpy as np


def generator(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def decaying(n: int, seed: int, rate: float = 0.05, symmetric: bool = False,
             scale: float = 1.0) -> np.ndarray:
    """|a_ij| ~ scale * exp(-rate |i - j|) with N(0,1) signs/magnitudes (Sec. 2 decay)."""
    g = generator(seed)
    a = g.standard_normal((n, n))
    i = np.arange(n)
    env = scale * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    a = a * env
    if symmetric:
        a = np.triu(a) + np.triu(a, 1).T
    return a


def block_scaled(alpha: np.ndarray, unit: np.ndarray) -> np.ndarray:
    """Matrix whose (i, k) 32x32 block is alpha[i, k] * unit."""
    nb = alpha.shape[0]
    b = unit.shape[0]
    out = np.zeros((nb * b, nb * b), dtype=np.float64)
    for i in range(nb):
        for k in range(nb):
            out[i * b:(i + 1) * b, k * b:(k + 1) * b] = alpha[i, k] * unit
    return out


def unit_block(seed: int, size: int = 32) -> np.ndarray:
    """A random size x size block with Frobenius norm exactly a power of two times 1.

    The entries are integers / 2^m chosen so that the sum of squares is an
    exact square of a power of two: every entry is +-1/32, so the Frobenius
    norm is exactly 1 (32*32 entries of square 1/1024).
    """
    g = generator(seed)
    return g.choice([-1.0, 1.0], size=(size, size)) / float(size)


def random_symmetric_with_gap(n: int, n_occ: int, seed: int, gap: float = 1.0) -> np.ndarray:
    """Symmetric matrix with a spectral gap of `gap` after the n_occ lowest eigenvalues."""
    g = generator(seed)
    q, _ = np.linalg.qr(g.standard_normal((n, n)))
    lo = -1.0 - g.uniform(0.0, 1.0, size=n_occ)
    hi = -1.0 + gap + g.uniform(0.0, 1.0, size=n - n_occ)
    ev = np.concatenate([lo, hi])
    a = (q * ev) @ q.T
    return 0.5 * (a + a.T)
