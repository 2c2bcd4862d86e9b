"""Seeded synthetic inputs shaped like the paper's water-cluster matrices.

Shared by the oracle, the tests and the benchmark; it contains no part of the
SpAMM or SP2 arithmetic.
"""
from .cluster import (BASIS_PER_MOLECULE, OCC_PER_MOLECULE, Request, WaterCluster,
                      lattice_sites, molecule_centres, request_seed, request_stream,
                      water_cluster)
from .cluster_torch import water_cluster_torch
from .hilbert import hilbert_index, transpose_index

__all__ = ["BASIS_PER_MOLECULE", "OCC_PER_MOLECULE", "Request", "WaterCluster",
           "lattice_sites", "molecule_centres", "request_seed", "request_stream",
           "water_cluster", "water_cluster_torch", "hilbert_index", "transpose_index"]
