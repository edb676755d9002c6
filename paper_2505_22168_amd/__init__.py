"""MI355X-native GMNN energy/force library (HIP kernels for gfx950 behind a
C ABI, include/gmnn.h).  This package is the thin Python binding: torch
tensors hold the device buffers; every step of the path runs in libgmnn.so.
Importing the package does not touch the GPU; the library is loaded on first
use and a missing build raises ImportError (there is no CPU fallback)."""
from ._capi import GMNNError, load as load_library, LIB_PATH
from .api import (System, NeighborList, Model, Outputs, EnergyForces, build_neighbors, energy_forces, MD,
                  maxwell_boltzmann, param_grads, EnergyForcesFunction, PARAM_NAMES,
                  estimate_capacity, last_layer_features, select_max_distance, LossSpec, ensemble_loss,
                  lr_factor, Adam, EnsembleTrainer)

__all__ = ["GMNNError", "load_library", "LIB_PATH", "System", "NeighborList", "Model", "Outputs", "MD",
           "maxwell_boltzmann", "param_grads", "EnergyForcesFunction", "PARAM_NAMES",
           "EnergyForces", "build_neighbors", "energy_forces", "estimate_capacity", "last_layer_features",
           "select_max_distance", "LossSpec", "ensemble_loss", "lr_factor", "Adam", "EnsembleTrainer"]
