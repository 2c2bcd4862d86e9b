"""Checks of the seeded input generators (shape, structure, determinism)."""
import numpy as np
import pytest

from watergen import hilbert_index, lattice_sites, request_stream, water_cluster


@pytest.mark.parametrize("ndim,bits", [(2, 4), (3, 3)])
def test_hilbert_curve_is_a_continuous_bijection(ndim, bits):
    side = 1 << bits
    grid = np.stack(np.meshgrid(*[np.arange(side)] * ndim, indexing="ij"), -1).reshape(-1, ndim)
    h = hilbert_index(grid, bits)
    assert sorted(h.tolist()) == list(range(side ** ndim))
    path = grid[np.argsort(h)]
    assert np.all(np.abs(np.diff(path, axis=0)).sum(axis=1) == 1)
    assert np.all(path[0] == 0)


def test_lattice_sites_nearest_first():
    s = lattice_sites(7)
    assert np.all(s[0] == 0)
    assert sorted(map(tuple, s[1:])) == sorted([(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),
                                                 (0, 0, -1), (0, 0, 1)])
    r2 = (lattice_sites(200) ** 2).sum(axis=1)
    assert np.all(np.diff(r2) >= 0)


def test_water_cluster_structure_and_determinism():
    w = water_cluster(30, 1.5, 0)
    assert w.n == 750 and w.n_occ == 150
    assert np.array_equal(w.f, w.f.T)
    d = np.diag(w.f)
    assert np.all(d.reshape(30, 25)[:, :5] == -1.0) and np.all(d.reshape(30, 25)[:, 5:] == 1.0)
    w2 = water_cluster(30, 1.5, 0)
    assert np.array_equal(w.f, w2.f)
    w3 = water_cluster(30, 1.5, 1)
    assert not np.array_equal(w.f, w3.f)
    # Jitter bounded by 0.3 A around 3.1 A lattice sites.
    q = w.centres / 3.1
    assert np.all(np.abs(q - np.round(q)) * 3.1 <= 0.3 + 1e-12)
    # Off-diagonal envelope: |F_ij| / (0.3 exp(-d/1.5)) is a |N(0,1)| sample.
    i, j = 3, 700
    dist = np.linalg.norm(w.centres[i // 25] - w.centres[j // 25])
    assert abs(w.f[i, j]) < 0.3 * np.exp(-dist / 1.5) * 8


def test_hilbert_ordering_keeps_neighbours_close():
    w = water_cluster(150, 1.5, 0)
    steps = np.linalg.norm(np.diff(w.centres, axis=0), axis=1)
    assert np.median(steps) < 3.1 * 1.5


def test_request_stream():
    r = request_stream(256, 20.0, seed=0)
    assert len(r) == 256 and r[0].arrival_s == 0.0
    assert all(30 <= q.molecules <= 400 and 1.2 <= q.decay <= 2.5 and q.tau in (1e-6, 1e-5)
               for q in r)
    arr = np.array([q.arrival_s for q in r])
    assert np.all(np.diff(arr) >= 0)
    assert 8.0 < arr[-1] < 20.0      # mean gap 50 ms
    assert [q.seed for q in r] == [q.seed for q in request_stream(256, 20.0, seed=0)]


def test_device_generator_follows_the_same_recipe():
    """The torch generator (run here on the CPU device) builds the same kind
    of matrix: exactly symmetric, diagonal -1 / +1 by orbital, the same
    centres, and off-diagonal magnitudes following 0.3 exp(-d / decay)."""
    import torch
    from watergen import water_cluster_torch
    f, n_occ = water_cluster_torch(12, 1.7, 5, device="cpu")
    w = water_cluster(12, 1.7, 5)
    f = f.numpy()
    assert f.shape == w.f.shape and n_occ == w.n_occ
    assert np.array_equal(f, f.T)
    assert np.array_equal(np.diag(f), np.diag(w.f))
    # Per molecule pair, the RMS of the 25 x 25 block is 0.3 exp(-d / decay)
    # up to sampling noise (625 normals); the same holds for numpy's draws.
    d = np.linalg.norm(w.centres[:, None] - w.centres[None], axis=2)
    env = 0.3 * np.exp(-d / 1.7)
    blocks = f.reshape(12, 25, 12, 25).transpose(0, 2, 1, 3)
    off = ~np.eye(12, dtype=bool)
    rms = np.sqrt((blocks ** 2).mean(axis=(2, 3)))[off]
    assert np.allclose(rms / env[off], 1.0, atol=0.2)
    # Deterministic per seed.
    g, _ = water_cluster_torch(12, 1.7, 5, device="cpu")
    assert np.array_equal(g.numpy(), f)
