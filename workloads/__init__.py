"""Seeded synthetic inputs for the GMNN energy/force path.

This package produces inputs only: periodic structures (positions, species,
cells, pbc flags) and model parameters drawn from a seed.  It holds none of the
method's arithmetic (no radial basis, moments, contractions or network), so
both the FP64 oracle and the GPU path may consume what it produces.
"""
from .structures import Batch, random_box, jittered_lattice, make_batch, species_counts, cluster_cut
from .configs import ModelSpec, ModelParams, WorkloadSpec, WORKLOADS, make_params, make_workload

__all__ = [
    "Batch", "random_box", "jittered_lattice", "make_batch", "species_counts", "cluster_cut",
    "ModelSpec", "ModelParams", "WorkloadSpec", "WORKLOADS", "make_params", "make_workload",
]
