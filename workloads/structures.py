"""Seeded periodic structures (inputs only; no model arithmetic).

Every generator draws from ``numpy.random.default_rng(seed)`` so a given seed
always produces the same positions, species and cells.  Positions are stored
as float32 (the precision the GPU path takes), cells as float64 with lattice
vectors as rows.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Batch:
    """A ragged batch of periodic structures, concatenated atom-wise.

    pos      [N,3]   float32  Cartesian positions in Angstrom
    species  [N]     int32    species index in [0, n_species)
    cell     [B,3,3] float64  lattice vectors as rows, Angstrom
    pbc      [B,3]   uint8    1 where the structure is periodic along that axis
    atom_ptr [B+1]   int64    structure b owns atoms atom_ptr[b]:atom_ptr[b+1]
    """

    pos: np.ndarray
    species: np.ndarray
    cell: np.ndarray
    pbc: np.ndarray
    atom_ptr: np.ndarray

    @property
    def n_atoms(self) -> int:
        return int(self.atom_ptr[-1])

    @property
    def n_structs(self) -> int:
        return int(self.cell.shape[0])

    def struct_of_atom(self) -> np.ndarray:
        counts = np.diff(self.atom_ptr)
        return np.repeat(np.arange(self.n_structs, dtype=np.int32), counts)

    def structure(self, b: int) -> "Batch":
        a0, a1 = int(self.atom_ptr[b]), int(self.atom_ptr[b + 1])
        return Batch(self.pos[a0:a1].copy(), self.species[a0:a1].copy(),
                     self.cell[b:b + 1].copy(), self.pbc[b:b + 1].copy(),
                     np.array([0, a1 - a0], dtype=np.int64))


def species_counts(n: int, ratio) -> np.ndarray:
    """Largest-remainder split of n atoms according to an integer ratio."""
    ratio = np.asarray(ratio, dtype=np.float64)
    exact = n * ratio / ratio.sum()
    base = np.floor(exact).astype(np.int64)
    rem = n - int(base.sum())
    order = np.argsort(-(exact - base), kind="stable")
    base[order[:rem]] += 1
    return base


def _assign_species(rng, n, ratio) -> np.ndarray:
    counts = species_counts(n, ratio)
    sp = np.repeat(np.arange(len(counts), dtype=np.int32), counts)
    return sp[rng.permutation(n)].astype(np.int32)


def _min_image_dist2(x: np.ndarray, others: np.ndarray, box: float) -> np.ndarray:
    d = others - x
    d -= box * np.round(d / box)
    return np.einsum("ij,ij->i", d, d)


def random_box(rng, n: int, box: float, ratio, min_sep: float = 0.9,
               relax_sweeps: int = 0, step: float = 0.1):
    """Cubic periodic box of side ``box`` filled by random sequential addition.

    Candidates closer than ``min_sep`` to an already placed atom (closest
    periodic image; every box used here is wider than 2*min_sep) are rejected.
    ``relax_sweeps`` random-walk sweeps follow: each atom in turn proposes a
    Gaussian step of width ``step`` that is accepted iff it keeps the minimum
    separation.  Returns (pos float32 [n,3], species int32 [n]).
    """
    pos = np.zeros((n, 3), dtype=np.float64)
    placed = 0
    tries = 0
    ms2 = min_sep * min_sep
    while placed < n:
        tries += 1
        if tries > 1000 * n + 10000:
            raise RuntimeError("random sequential addition did not converge")
        c = rng.random(3) * box
        if placed and _min_image_dist2(c, pos[:placed], box).min() < ms2:
            continue
        pos[placed] = c
        placed += 1
    for _ in range(relax_sweeps):
        for i in range(n):
            c = pos[i] + rng.normal(0.0, step, 3)
            c -= box * np.floor(c / box)
            d2 = _min_image_dist2(c, pos, box)
            d2[i] = np.inf
            if d2.min() >= ms2:
                pos[i] = c
    species = _assign_species(rng, n, ratio)
    return pos.astype(np.float32), species


def jittered_lattice(rng, reps, a: float, ratio, jitter: float):
    """Simple-cubic lattice of reps[0]*reps[1]*reps[2] sites, spacing ``a``,
    with i.i.d. Gaussian jitter of width ``jitter`` on every coordinate.
    Returns (pos float32 [n,3], species int32 [n], box lengths [3])."""
    nx, ny, nz = reps
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    pos = g.reshape(-1, 3).astype(np.float64) * a
    pos += rng.normal(0.0, jitter, pos.shape)
    box = np.array([nx * a, ny * a, nz * a])
    pos -= box * np.floor(pos / box)
    species = _assign_species(rng, pos.shape[0], ratio)
    return pos.astype(np.float32), species, box


def make_batch(structs) -> Batch:
    """Concatenate a list of (pos, species, cell[3,3], pbc[3]) tuples."""
    pos = np.concatenate([s[0] for s in structs]).astype(np.float32)
    species = np.concatenate([s[1] for s in structs]).astype(np.int32)
    cell = np.stack([np.asarray(s[2], dtype=np.float64) for s in structs])
    pbc = np.stack([np.asarray(s[3], dtype=np.uint8) for s in structs])
    ptr = np.zeros(len(structs) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(s[1]) for s in structs])
    return Batch(pos, species, cell, pbc, ptr)


def cluster_cut(batch: Batch, center: int, radius: float):
    """Non-periodic cluster of the atoms of ``center``'s structure whose closest
    periodic image lies within ``radius`` of atom ``center``, each placed at
    that image.  Needs every periodic cell width above 2 * radius (one image
    per atom).

    Positions are float64: centre position + (x_j - x_c + S h), evaluated in
    float64 from the float32 inputs, so every separation inside the cluster
    equals the periodic one to float64 rounding.  Returns (Batch, index of each
    cluster atom in ``batch``, its distance from the centre); the centre is
    cluster atom 0.

    Input manipulation only.  With a finite cutoff r_c, an atom's energy
    depends on atoms within r_c of it and an atom's force on atoms within
    2 r_c, so cluster atoms within radius - r_c of the centre have their
    periodic energies and those within radius - 2 r_c their periodic forces.
    """
    soa = batch.struct_of_atom()
    b = int(soa[center])
    a0, a1 = int(batch.atom_ptr[b]), int(batch.atom_ptr[b + 1])
    h = batch.cell[b]
    x = batch.pos[a0:a1].astype(np.float64)
    xc = x[center - a0]
    frac = (x - xc) @ np.linalg.inv(h)
    S = -np.round(frac) * batch.pbc[b].astype(np.float64)
    d = (x - xc) + S @ h
    dist = np.sqrt((d * d).sum(1))
    keep = np.nonzero(dist < radius)[0]
    keep = np.concatenate([[center - a0], keep[keep != center - a0]])
    pos = xc + d[keep]
    cut = Batch(pos, batch.species[a0:a1][keep].copy(), h[None].copy(), np.zeros((1, 3), dtype=np.uint8),
                np.array([0, keep.size], dtype=np.int64))
    return cut, keep + a0, dist[keep]
