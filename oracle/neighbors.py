"""Brute-force periodic neighbour list (oracle; test infrastructure only).

Definition (Section 2.1, the moment sum runs over all neighbours j != i of
atom i; Section 3.5, small periodic cells need several images of one
neighbour): the list holds every triple (i, j, S) with S an integer image
vector such that the separation

    d = x_j - x_i + S . h          (h: lattice vectors as rows)

satisfies |d| < r_c, except the atom itself (i, i, 0).  Images of the atom
itself (i, i, S != 0) are kept.  S is relative to the positions as given
(they need not lie inside the cell).  Non-periodic axes only take S = 0.

Inclusion test (reading; the paper does not fix a precision): the float32
input coordinates are widened to float64 and

    dx = (x_j - x_i) + ((Sx*h[0,0] + Sy*h[1,0]) + Sz*h[2,0])    (same for y, z)
    d2 = (dx*dx + dy*dy) + dz*dz,   accepted iff d2 < rc*rc

with rc the float32 cutoff widened to float64, each operation rounded once
(no fused multiply-add).  A pair with d2 == 0 (coincident atoms) is reported
separately and left out of the list.

Order (canonical): rows by i; inside a row by (j, Sx, Sy, Sz) ascending.
This is a plain enumeration of every image vector in a range wide enough to
contain all candidates; it is O(N^2 * images) and meant for small inputs or
for sampled rows.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np


@dataclass
class NeighborList:
    i: np.ndarray        # [P] int64, row (centre atom, global index)
    j: np.ndarray        # [P] int64, neighbour atom (global index)
    S: np.ndarray        # [P,3] int64, image vector
    coincident: int = 0  # number of (i, j, S) with zero separation

    @property
    def n_pairs(self) -> int:
        return int(self.i.shape[0])

    def row_ptr(self, n_atoms: int) -> np.ndarray:
        ptr = np.zeros(n_atoms + 1, dtype=np.int64)
        np.add.at(ptr, self.i + 1, 1)
        return np.cumsum(ptr)


def _image_range(cell: np.ndarray, pbc, rc: float):
    """Per-axis half-width of the image window around S0 = -round(f_j - f_i):
    a listed pair has |f_j - f_i + S|_k < rc / width_k (width: distance
    between the two cell faces normal to axis k) and |f_j - f_i + S0|_k <= 1/2,
    so |S - S0|_k <= ceil(rc / width_k + 1/2)."""
    vol = abs(float(np.linalg.det(cell)))
    n = []
    for k in range(3):
        if not pbc[k]:
            n.append(0)
            continue
        a, b = cell[(k + 1) % 3], cell[(k + 2) % 3]
        width = vol / float(np.linalg.norm(np.cross(a, b)))
        n.append(int(math.ceil(rc / width + 0.5 + 1e-9)))
    return n


def _structure_pairs(pos32: np.ndarray, cell: np.ndarray, pbc, cutoff32: float, rows=None):
    n = pos32.shape[0]
    x = pos32.astype(np.float64)
    rc = float(np.float64(np.float32(cutoff32)))
    rc2 = rc * rc
    inv = np.linalg.inv(cell)
    frac = x @ inv
    nr = _image_range(cell, pbc, rc)
    rng = [np.arange(-m, m + 1) for m in nr]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out_i, out_j, out_S = [], [], []
    coincident = 0
    pbc_mask = np.array([1.0 if p else 0.0 for p in pbc])
    for i in rows:
        # centre of the image window for every j: S0 = -round(f_j - f_i) on periodic axes
        S0 = -np.round(frac - frac[i]) * pbc_mask          # [n,3]
        S0 = S0.astype(np.int64)
        grid = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)  # [M,3]
        S = S0[:, None, :] + grid[None, :, :]                # [n,M,3]
        Sf = S.astype(np.float64)
        dx = [None, None, None]
        for c in range(3):
            sh = (Sf[..., 0] * cell[0, c] + Sf[..., 1] * cell[1, c]) + Sf[..., 2] * cell[2, c]
            dx[c] = (x[:, c][:, None] - x[i, c]) + sh
        d2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2]
        self_img = (np.arange(n)[:, None] == i) & np.all(S == 0, axis=-1)
        keep = (d2 < rc2) & ~self_img
        zero = keep & (d2 == 0.0)
        coincident += int(zero.sum())
        keep &= ~zero
        jj, mm = np.nonzero(keep)
        SS = S[jj, mm]
        order = np.lexsort((SS[:, 2], SS[:, 1], SS[:, 0], jj))
        out_i.append(np.full(len(order), i, dtype=np.int64))
        out_j.append(jj[order].astype(np.int64))
        out_S.append(SS[order].astype(np.int64))
    if out_i:
        return np.concatenate(out_i), np.concatenate(out_j), np.concatenate(out_S), coincident
    e = np.zeros(0, dtype=np.int64)
    return e, e, np.zeros((0, 3), dtype=np.int64), coincident


def brute_force_neighbors(batch, cutoff: float, rows=None) -> NeighborList:
    """All (i, j, S) of every structure in ``batch`` (workloads.Batch), with
    global atom indices, in canonical order.  ``rows`` (global atom indices,
    ascending) restricts the enumeration to those centre atoms."""
    ii, jj, SS = [], [], []
    coincident = 0
    for b in range(batch.n_structs):
        a0, a1 = int(batch.atom_ptr[b]), int(batch.atom_ptr[b + 1])
        sub_rows = None
        if rows is not None:
            r = np.asarray(rows)
            r = r[(r >= a0) & (r < a1)]
            if r.size == 0:
                continue
            sub_rows = r - a0
        i, j, S, c = _structure_pairs(batch.pos[a0:a1], batch.cell[b], batch.pbc[b], cutoff, sub_rows)
        ii.append(i + a0)
        jj.append(j + a0)
        SS.append(S)
        coincident += c
    if not ii:
        e = np.zeros(0, dtype=np.int64)
        return NeighborList(e, e, np.zeros((0, 3), dtype=np.int64), coincident)
    return NeighborList(np.concatenate(ii), np.concatenate(jj), np.concatenate(SS), coincident)
