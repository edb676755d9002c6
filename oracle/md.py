"""Velocity-Verlet NVE integration with oracle forces (test infrastructure
only).  Section 3.5 of the paper runs MD with the model's forces; the
integrator is the textbook velocity Verlet:

    v(t + dt/2) = v(t) + dt/2 a(t)
    x(t + dt)   = x(t) + dt v(t + dt/2)
    v(t + dt)   = v(t + dt/2) + dt/2 a(t + dt),     a = k_u F / m

with F in eV/A, m in amu, dt in fs, v in A/fs and k_u = 9.648533e-3
A fs^-2 per eV/(A amu) (1 amu A^2 fs^-2 = 103.6427 eV).  The neighbour list
is rebuilt from scratch at every step (no skin), in float64.
"""
from __future__ import annotations

import numpy as np

from .gmnn import evaluate
from .neighbors import brute_force_neighbors

ACCEL_UNIT = 9.648533e-3


def _forces(batch, params, x, udd=None):
    """Forces and potential energy at x; udd = (A, B) adds the
    uncertainty-driven bias of Section 2.3 (eq. udd) to the potential."""
    from workloads import Batch
    b = Batch(x.astype(np.float32), batch.species, batch.cell, batch.pbc, batch.atom_ptr)
    nl = brute_force_neighbors(b, params.spec.r_cut)
    # evaluate at the float64 positions (the list decisions use float32)
    import torch
    from .gmnn import atomic_energies, udd_bias
    pos = torch.as_tensor(x).requires_grad_(True)
    Ei = atomic_energies(b, params, nl, pos=pos)
    E = Ei.mean(1).sum()
    if udd is not None:
        soa = torch.as_tensor(b.struct_of_atom(), dtype=torch.long)
        Eb = torch.zeros((b.n_structs, Ei.shape[1]), dtype=Ei.dtype).index_add(0, soa, Ei)
        nb = torch.as_tensor(np.diff(b.atom_ptr), dtype=Ei.dtype)
        E = E + udd_bias(Eb, nb, udd[0], udd[1]).sum()
    (g,) = torch.autograd.grad(E, pos)
    return -g.numpy(), float(E.detach())


def velocity_verlet(batch, params, x0, v0, masses, dt, n_steps, udd=None):
    """Positions, velocities and potential energies after each step (float64)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    v = np.asarray(v0, dtype=np.float64).copy()
    inv_m = 1.0 / np.asarray(masses, dtype=np.float64)[:, None]
    F, E = _forces(batch, params, x, udd)
    xs, vs, es = [], [], []
    for _ in range(n_steps):
        v = v + 0.5 * dt * ACCEL_UNIT * F * inv_m
        x = x + dt * v
        F, E = _forces(batch, params, x, udd)
        v = v + 0.5 * dt * ACCEL_UNIT * F * inv_m
        xs.append(x.copy())
        vs.append(v.copy())
        es.append(E)
    return np.array(xs), np.array(vs), np.array(es)


def kinetic_energy(v, masses):
    return float(0.5 * (np.asarray(masses)[:, None] * v * v).sum() / ACCEL_UNIT)
