"""Water-cluster-shaped Fock matrices generated on a torch device.

The same recipe as `cluster.water_cluster` (molecule centres, Hilbert
order, 25 basis functions per molecule, diagonal -1 / +1, off-diagonal
0.3 g_ij exp(-d_ij / decay) mirrored from the strict upper triangle), with
the N x N standard normals drawn by torch's generator on the device instead
of numpy's PCG64, so that serving streams of many large requests can be
built in device memory in milliseconds.  The centres come from numpy exactly
as in `water_cluster`; the matrices themselves differ from `water_cluster`'s
for the same seed (a different random stream), not in distribution.

This module holds no SpAMM or SP2 arithmetic.
"""
from __future__ import annotations

import numpy as np

from .cluster import (BASIS_PER_MOLECULE, COUPLING, OCC_PER_MOLECULE, WaterCluster,
                      molecule_centres)


def water_cluster_torch(molecules: int, decay: float = 1.5, seed: int = 0, device="cuda"):
    """(F as a float64 torch tensor on `device`, n_occ)."""
    import torch
    if decay <= 0:
        raise ValueError("decay length must be positive")
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = molecule_centres(molecules, rng)
    nb = BASIS_PER_MOLECULE
    n = molecules * nb
    d = np.linalg.norm(centres[:, None, :] - centres[None, :, :], axis=2)
    env = torch.from_numpy(COUPLING * np.exp(-d / decay)).to(device)
    env = env.repeat_interleave(nb, dim=0).repeat_interleave(nb, dim=1)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    g = torch.randn((n, n), generator=gen, dtype=torch.float64, device=device)
    f = torch.triu(g * env, diagonal=1)
    del g, env
    f = f + f.T
    occ = (torch.arange(n, device=device) % nb) < OCC_PER_MOLECULE
    f.diagonal().copy_(torch.where(occ, -1.0, 1.0).to(torch.float64))
    return f, OCC_PER_MOLECULE * molecules


__all__ = ["water_cluster_torch", "WaterCluster"]
