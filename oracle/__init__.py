"""FP64 CPU oracle for the GMNN energy/force path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path:
it is a plain, slow, direct transcription of the method's definitions
(Section 2.1 of the paper: additive energy, Gaussian radial basis with
species-pair coefficients, Cartesian moments, full tensor contractions,
network readout with per-element scale and shift; Section 3.3: forces and
virials as gradients; Section 2.2: shallow-ensemble statistics; Section
2.3: the uncertainty-driven bias; Section 2.4: last-layer gradient features
and greedy maximum-distance selection; Section 2.1's Bessel-like basis as an
alternative to the Gaussians; Section 2.2's probabilistic losses with
Section 3.4's loss terms, Adam parameter groups and learning-rate
schedules).

Every function here is pinned by tests under tests/ against closed forms,
invariances, brute force or finite differences; none is "parity unpinned".
"""
from .neighbors import brute_force_neighbors, NeighborList
from .bal import last_layer_features, max_distance_selection
from .ensemble_training import (
    LossSpec, ensemble_loss, ensemble_loss_grads, ensemble_loss_and_param_grads, adam_step, lr_factor,
)
from .gmnn import (
    radial_basis, cutoff_fn, pair_vectors, moments, invariants, feature_index,
    mlp, atomic_energies, evaluate, OracleResult, loss_and_param_grads, udd_bias, evaluate_udd, UddResult,
)

__all__ = [
    "brute_force_neighbors", "NeighborList", "radial_basis", "cutoff_fn", "pair_vectors",
    "moments", "invariants", "feature_index", "mlp", "atomic_energies", "evaluate",
    "OracleResult", "loss_and_param_grads", "udd_bias", "evaluate_udd", "UddResult",
    "last_layer_features", "max_distance_selection",
    "LossSpec", "ensemble_loss", "ensemble_loss_grads", "ensemble_loss_and_param_grads", "adam_step", "lr_factor",
]
