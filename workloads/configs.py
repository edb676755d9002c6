"""The five synthetic workloads and seeded model parameters (inputs only).

Hyperparameters that the paper leaves open are fixed here as readings:
  * basis centres r_min + k*delta, delta = (r_cut - r_min)/(K-1), r_min = 0.5 A,
    Gaussian width gamma = 1/(2 delta^2);
  * moment prefactor psi_scale = n_ref^(-1/4), n_ref = round(rho * 4/3 * pi * r_cut^3)
    (the mean neighbour count), which keeps the invariants and the forces O(1)
    with unit output scale;
  * weights W ~ N(0, 1/fan_in), biases ~ N(0, 0.1^2), basis coefficients
    beta ~ N(0, 1), drawn in the order beta, W1, b1, W2, b2, W3, b3;
  * per-species scale sigma_z = sigma0 * (1 + z/4) and shift mu_z = -(z + 1) eV.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

from .structures import Batch, jittered_lattice, make_batch, random_box


@dataclass(frozen=True)
class ModelSpec:
    n_species: int
    r_cut: float = 5.0
    n_radial: int = 5          # S
    n_basis: int = 7           # K
    r_min: float = 0.5
    hidden: tuple = (32, 32)   # (H1, H2)
    n_heads: int = 1
    psi_scale: float = 49.0 ** -0.25
    sigma0: float = 1.0
    basis: str = "gaussian"    # radial basis: "gaussian" or "bessel"

    @property
    def delta(self) -> float:
        return (self.r_cut - self.r_min) / (self.n_basis - 1)

    @property
    def gamma(self) -> float:
        return 1.0 / (2.0 * self.delta * self.delta)

    @property
    def n_features(self) -> int:
        s = self.n_radial
        pairs = s * (s + 1) // 2
        triples_sym = s * (s + 1) * (s + 2) // 6
        return s + 3 * pairs + triples_sym + 2 * pairs * s + s ** 3


@dataclass
class ModelParams:
    spec: ModelSpec
    beta: np.ndarray      # [n_sp, n_sp, S, K]
    W1: np.ndarray        # [F, H1]
    b1: np.ndarray        # [H1]
    W2: np.ndarray        # [H1, H2]
    b2: np.ndarray        # [H2]
    W3: np.ndarray        # [H2, heads]
    b3: np.ndarray        # [heads]
    scale: np.ndarray     # [n_sp]
    shift: np.ndarray     # [n_sp]

    def as_dict(self):
        return {k: getattr(self, k) for k in ("beta", "W1", "b1", "W2", "b2", "W3", "b3", "scale", "shift")}

    def n_params(self) -> int:
        return int(sum(v.size for v in self.as_dict().values()))


def make_params(spec: ModelSpec, seed: int) -> ModelParams:
    rng = np.random.default_rng(seed)
    n_sp, S, K = spec.n_species, spec.n_radial, spec.n_basis
    F = spec.n_features
    H1, H2 = spec.hidden
    beta = rng.normal(0.0, 1.0, (n_sp, n_sp, S, K))
    W1 = rng.normal(0.0, 1.0 / math.sqrt(F), (F, H1))
    b1 = rng.normal(0.0, 0.1, H1)
    W2 = rng.normal(0.0, 1.0 / math.sqrt(H1), (H1, H2))
    b2 = rng.normal(0.0, 0.1, H2)
    W3 = rng.normal(0.0, 1.0 / math.sqrt(H2), (H2, spec.n_heads))
    b3 = rng.normal(0.0, 0.1, spec.n_heads)
    z = np.arange(n_sp, dtype=np.float64)
    scale = spec.sigma0 * (1.0 + 0.25 * z)
    shift = -(z + 1.0)
    return ModelParams(spec, beta, W1, b1, W2, b2, W3, b3, scale, shift)


def _n_ref(rho: float, rc: float) -> int:
    return int(round(rho * 4.0 / 3.0 * math.pi * rc ** 3))


@dataclass(frozen=True)
class WorkloadSpec:
    name: str
    description: str
    seed: int
    model: ModelSpec
    skin: float = 0.0


def _cubic(L):
    return np.eye(3) * L


def _c1(seed):
    rng = np.random.default_rng(seed)
    pos, sp = random_box(rng, 48, 8.0, (1, 2), min_sep=0.9)
    return make_batch([(pos, sp, _cubic(8.0), (1, 1, 1))])


def _c2(seed, n=1536, rho=0.1, sweeps=20):
    rng = np.random.default_rng(seed)
    L = (n / rho) ** (1.0 / 3.0)
    pos, sp = random_box(rng, n, L, (15, 8, 2, 1, 4), min_sep=0.9, relax_sweeps=sweeps, step=0.1)
    return make_batch([(pos, sp, _cubic(L), (1, 1, 1))])


def _ragged(seed, n_structs, n_lo, n_hi, ratio, rho=0.1):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, n_structs)
    structs = []
    for n in sizes:
        L = (n / rho) ** (1.0 / 3.0)
        pos, sp = random_box(rng, int(n), L, ratio, min_sep=0.9)
        structs.append((pos, sp, _cubic(L), (1, 1, 1)))
    return make_batch(structs)


def _c4(seed, reps=(50, 50, 40), rho=0.08):
    rng = np.random.default_rng(seed)
    a = (1.0 / rho) ** (1.0 / 3.0)
    pos, sp, box = jittered_lattice(rng, reps, a, (3, 1, 4), jitter=0.1)
    return make_batch([(pos, sp, np.diag(box), (1, 1, 1))])


# Output scale sigma0 of every workload.  With psi_scale = n_ref^(-1/4) the
# forces of the random-weight models are already O(1) eV/A, so sigma0 = 1.
SIGMA0 = {"tiny": 1.0, "liquid": 1.0, "train": 1.0, "solid": 1.0, "ensemble": 1.0}

WORKLOADS = {
    "tiny": WorkloadSpec(
        "tiny", "48-atom 8 A cubic box, 2 species 16:32, r_cut 5, MLP 2x32", 0,
        ModelSpec(n_species=2, r_cut=5.0, hidden=(32, 32), psi_scale=_n_ref(48 / 512.0, 5.0) ** -0.25,
                  sigma0=SIGMA0["tiny"])),
    "liquid": WorkloadSpec(
        "liquid", "1536-atom liquid-like box, 5 species 15:8:2:1:4, rho 0.1/A^3, r_cut 5, MLP 2x256", 1,
        ModelSpec(n_species=5, r_cut=5.0, hidden=(256, 256), psi_scale=_n_ref(0.1, 5.0) ** -0.25,
                  sigma0=SIGMA0["liquid"])),
    "train": WorkloadSpec(
        "train", "32 structures of 100-600 atoms, 5 species, rho 0.1/A^3, r_cut 5, MLP 2x512", 2,
        ModelSpec(n_species=5, r_cut=5.0, hidden=(512, 512), psi_scale=_n_ref(0.1, 5.0) ** -0.25,
                  sigma0=SIGMA0["train"])),
    "solid": WorkloadSpec(
        "solid", "100,000-atom jittered simple-cubic lattice, 3 species 3:1:4, rho 0.08/A^3, r_cut 6, skin 1, MLP 2x512", 3,
        ModelSpec(n_species=3, r_cut=6.0, hidden=(512, 512), psi_scale=_n_ref(0.08, 6.0) ** -0.25,
                  sigma0=SIGMA0["solid"]), skin=1.0),
    "ensemble": WorkloadSpec(
        "ensemble", "256 structures of 20-200 atoms, 4 species, rho 0.1/A^3, r_cut 5, MLP 2x256, 16 heads", 4,
        ModelSpec(n_species=4, r_cut=5.0, hidden=(256, 256), n_heads=16, psi_scale=_n_ref(0.1, 5.0) ** -0.25,
                  sigma0=SIGMA0["ensemble"])),
}


def make_workload(name: str, **overrides) -> tuple[Batch, ModelParams, WorkloadSpec]:
    """Structures and parameters of a named workload.  ``overrides`` shrink the
    structure generator for tests (e.g. n=200 for the liquid box,
    n_structs=4 for ragged batches, reps=(8,8,6) for the lattice)."""
    spec = WORKLOADS[name]
    if name == "tiny":
        batch = _c1(spec.seed)
    elif name == "liquid":
        batch = _c2(spec.seed, **overrides)
    elif name == "train":
        kw = dict(n_structs=32, n_lo=100, n_hi=600)
        kw.update(overrides)
        batch = _ragged(spec.seed, ratio=(15, 8, 2, 1, 4), **kw)
    elif name == "solid":
        batch = _c4(spec.seed, **overrides)
    elif name == "ensemble":
        kw = dict(n_structs=256, n_lo=20, n_hi=200)
        kw.update(overrides)
        batch = _ragged(spec.seed, ratio=(1, 1, 1, 1), **kw)
    else:
        raise KeyError(name)
    params = make_params(spec.model, spec.seed + 1000)
    return batch, params, spec
