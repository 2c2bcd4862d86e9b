"""Seeded synthetic water-cluster-shaped Fock matrices.

The paper's inputs are FreeON B3LYP/6-31G** Fockians of water clusters:
25 basis functions per molecule, five doubly occupied orbitals per molecule,
atoms ordered along a Hilbert curve (Sec. 4).  Those matrices are not
available, so this module builds matrices with the same shape, the same
per-molecule structure and the same exponential decay with distance
(Sec. 2, matrices with decay):

* molecule centres: the M sites of a cubic lattice (3.1 A spacing) nearest
  the origin, ties broken lexicographically, each coordinate jittered by
  U(-0.3, 0.3) A;
* molecules ordered by the 3-D Hilbert index of their centres on a 2^10 grid
  spanning the bounding box;
* 25 basis functions per molecule, all at the molecule centre; functions 0-4
  are occupied (F_ii = -1), functions 5-24 virtual (F_ii = +1);
* F_ij = 0.3 * g_ij * exp(-d_ij / decay) for i != j, g_ij ~ N(0, 1) drawn for
  i < j and mirrored, d_ij the distance between the two molecule centres
  (0 inside a molecule).  Nothing is truncated.

n_occ = 5 M.  Random draws, in order: the jitter (M x 3 uniforms), then one
standard normal per entry of an N x N row-major array whose strict upper
triangle is used.

This module holds no SpAMM or SP2 arithmetic; it is the one input source
shared by the oracle and the device path.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

from .hilbert import hilbert_index

BASIS_PER_MOLECULE = 25
OCC_PER_MOLECULE = 5
LATTICE_SPACING = 3.1     # Angstrom
JITTER = 0.3              # Angstrom, half-width of the uniform jitter
COUPLING = 0.3            # prefactor of the off-diagonal entries
HILBERT_BITS = 10


@dataclasses.dataclass
class WaterCluster:
    f: np.ndarray            # [n, n] float64, symmetric
    n_occ: int
    centres: np.ndarray      # [M, 3] Angstrom, in Hilbert order
    molecules: int
    decay: float
    seed: int

    @property
    def n(self) -> int:
        return self.f.shape[0]


def lattice_sites(m: int) -> np.ndarray:
    """The m integer lattice sites nearest the origin, ordered by (r^2, x, y, z)."""
    if m < 1:
        raise ValueError("need at least one molecule")
    r = int(np.ceil((3.0 * m / (4.0 * np.pi)) ** (1.0 / 3.0))) + 3
    ax = np.arange(-r, r + 1)
    x, y, z = np.meshgrid(ax, ax, ax, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    r2 = (pts ** 2).sum(axis=1)
    order = np.lexsort((pts[:, 2], pts[:, 1], pts[:, 0], r2))
    return pts[order[:m]]


def hilbert_order(centres: np.ndarray, bits: int = HILBERT_BITS) -> np.ndarray:
    """Permutation that sorts points by Hilbert index over their bounding box."""
    lo = centres.min(axis=0)
    span = centres.max(axis=0) - lo
    extent = float(span.max()) if span.size else 0.0
    cells = 1 << bits
    if extent <= 0.0:
        q = np.zeros(centres.shape, dtype=np.int64)
    else:
        q = np.floor((centres - lo) / extent * (cells - 1) + 0.5).astype(np.int64)
        q = np.clip(q, 0, cells - 1)
    h = hilbert_index(q, bits)
    return np.argsort(h, kind="stable")


def molecule_centres(m: int, rng: np.random.Generator) -> np.ndarray:
    sites = lattice_sites(m).astype(np.float64) * LATTICE_SPACING
    sites += rng.uniform(-JITTER, JITTER, size=sites.shape)
    return sites[hilbert_order(sites)]


def water_cluster(molecules: int, decay: float = 1.5, seed: int = 0,
                  row_chunk: int = 512) -> WaterCluster:
    """Build the synthetic Fockian of `molecules` water-like molecules."""
    if decay <= 0:
        raise ValueError("decay length must be positive")
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = molecule_centres(molecules, rng)
    nb = BASIS_PER_MOLECULE
    n = molecules * nb
    mol_of = np.arange(n) // nb
    f = np.zeros((n, n), dtype=np.float64)
    for r0 in range(0, n, row_chunk):
        r1 = min(n, r0 + row_chunk)
        g = rng.standard_normal((r1 - r0, n))
        d = np.linalg.norm(centres[mol_of[r0:r1], None, :] - centres[None, :, :], axis=2)
        env = COUPLING * np.exp(-d / decay)               # [rows, M]
        vals = g * np.repeat(env, nb, axis=1)             # [rows, n]
        rows = np.arange(r0, r1)
        upper = np.arange(n)[None, :] > rows[:, None]
        f[r0:r1] = np.where(upper, vals, 0.0)
    # Mirror the strict upper triangle tile by tile (no full-size temporaries).
    t = 1024
    for i0 in range(0, n, t):
        i1 = min(n, i0 + t)
        for j0 in range(0, i1, t):
            j1 = min(n, j0 + t)
            blk = f[j0:j1, i0:i1].T.copy()
            if j0 == i0:
                low = np.tril(np.ones((i1 - i0, j1 - j0), dtype=bool), -1)
                f[i0:i1, j0:j1][low] = blk[low]
            else:
                f[i0:i1, j0:j1] = blk
    diag = np.where((np.arange(n) % nb) < OCC_PER_MOLECULE, -1.0, 1.0)
    f[np.arange(n), np.arange(n)] = diag
    return WaterCluster(f=f, n_occ=OCC_PER_MOLECULE * molecules, centres=centres,
                        molecules=molecules, decay=float(decay), seed=int(seed))


def request_seed(stream_seed: int, index: int) -> int:
    """Per-request generator seed of a serving stream (stable across platforms)."""
    h = hashlib.sha256(f"{int(stream_seed)}:{int(index)}".encode()).digest()
    return int.from_bytes(h[:4], "little")


@dataclasses.dataclass
class Request:
    index: int
    arrival_s: float
    molecules: int
    decay: float
    tau: float
    seed: int


def request_stream(count: int = 256, rate_per_s: float = 20.0, seed: int = 0,
                   min_molecules: int = 30, max_molecules: int = 400,
                   decay_range=(1.2, 2.5), taus=(1e-6, 1e-5)) -> list[Request]:
    """Poisson arrival stream of SP2 requests of mixed size and decay."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    mols = rng.integers(min_molecules, max_molecules + 1, size=count)
    decays = rng.uniform(decay_range[0], decay_range[1], size=count)
    tau_pick = rng.integers(0, len(taus), size=count)
    return [Request(index=i, arrival_s=float(arrivals[i]), molecules=int(mols[i]),
                    decay=float(decays[i]), tau=float(taus[tau_pick[i]]),
                    seed=request_seed(seed, i)) for i in range(count)]
