"""Hilbert-curve index of integer points on a 2^bits grid.

Locality-preserving ordering of the molecules is a key ingredient of the
paper's workloads (Sec. 4, the basis is ordered along a Hilbert curve; Fig. 1
shows the resulting clustering of like magnitudes).  This module computes the
index with Skilling's transpose method (J. Skilling, "Programming the Hilbert
curve", AIP Conf. Proc. 707, 381 (2004)): the coordinates are turned in place
into the "transposed" Hilbert index by undoing the curve's reflections and
exchanges from the most significant bit down, Gray-encoding, and finally
interleaving the bits.

This is input-generation infrastructure: it holds none of the SpAMM or SP2
arithmetic and is shared by the oracle and the device path alike.
"""
from __future__ import annotations

import numpy as np


def transpose_index(coords: np.ndarray, bits: int) -> np.ndarray:
    """Skilling's axes-to-transpose map, vectorised over points.

    coords: int array [npts, ndim] with entries in [0, 2^bits).
    Returns the transposed index, same shape: bit b of the Hilbert index's
    digit for axis d is bit b of the returned column d.
    """
    x = np.array(coords, dtype=np.int64, copy=True)
    if x.ndim != 2:
        raise ValueError("coords must be [npts, ndim]")
    if bits < 1 or bits > 20:
        raise ValueError("bits out of range")
    if np.any(x < 0) or np.any(x >= (1 << bits)):
        raise ValueError("coordinate outside the grid")
    ndim = x.shape[1]
    top = 1 << (bits - 1)
    q = top
    # Undo the rotations/reflections, from the coarsest bit to the finest.
    while q > 1:
        p = q - 1
        for d in range(ndim):
            has = (x[:, d] & q) != 0
            # Where the bit is set: invert the low bits of axis 0.
            x[has, 0] ^= p
            # Elsewhere: exchange the low bits of axis 0 and axis d.
            nh = ~has
            t = (x[nh, 0] ^ x[nh, d]) & p
            x[nh, 0] ^= t
            x[nh, d] ^= t
        q >>= 1
    # Gray encode.
    for d in range(1, ndim):
        x[:, d] ^= x[:, d - 1]
    t = np.zeros(x.shape[0], dtype=np.int64)
    q = top
    while q > 1:
        t ^= np.where((x[:, ndim - 1] & q) != 0, q - 1, 0)
        q >>= 1
    for d in range(ndim):
        x[:, d] ^= t
    return x


def hilbert_index(coords: np.ndarray, bits: int) -> np.ndarray:
    """Scalar Hilbert index (int64) of each point; ndim*bits must be <= 62."""
    coords = np.asarray(coords)
    ndim = coords.shape[1]
    if ndim * bits > 62:
        raise ValueError("index does not fit in int64")
    tr = transpose_index(coords, bits)
    h = np.zeros(tr.shape[0], dtype=np.int64)
    # Interleave: most significant bit first, axis 0 first within a bit.
    for b in range(bits - 1, -1, -1):
        for d in range(ndim):
            h = (h << 1) | ((tr[:, d] >> b) & 1)
    return h
