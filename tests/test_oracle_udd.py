"""Pins of the oracle's uncertainty-driven bias (Section 2.3, eq. udd):
E_bias = A [exp(-var / (M N B^2)) - 1] on the head-energy variance.

* heads that differ by constant output offsets: the variance has a closed
  form (and does not depend on positions), so E_bias is known by hand and the
  biased forces equal the unbiased ones;
* forces are minus the finite-difference gradient of Ebar + E_bias;
* the force is sum_m c_m F^m with c_m = 1/M + E_bias'(var) 2 (E^m - Ebar)/M,
  checked against per-head forces from single-head models;
* A = 0 gives the unbiased evaluation."""
import copy
import dataclasses
import math

import numpy as np

from oracle import brute_force_neighbors, evaluate, evaluate_udd
from workloads import make_workload

A, B = 1.0, 1.2


def _ens(n_structs=2, **kw):
    batch, params, spec = make_workload("ensemble", n_structs=n_structs, **kw)
    return batch, params, brute_force_neighbors(batch, 5.0)


def test_constant_head_offsets_closed_form():
    batch, params, nl = _ens()
    p = copy.deepcopy(params)
    M = p.spec.n_heads
    p.W3 = np.repeat(p.W3[:, :1], M, 1)
    offs = np.linspace(-0.3, 0.3, M)
    p.b3 = p.b3[0] + offs
    r = evaluate_udd(batch, p, nl, A, B)
    sp = batch.species
    for b in range(batch.n_structs):
        a0, a1 = batch.atom_ptr[b], batch.atom_ptr[b + 1]
        ssum = p.scale[sp[a0:a1]].sum()
        var = offs.var() * ssum ** 2            # E^m = E^0 + offs_m sum_i sigma_i
        n = a1 - a0
        want = A * (math.exp(-var / (M * n * B * B)) - 1.0)
        assert abs(r.bias_energy[b] - want) < 1e-12 * max(1.0, abs(want))
        assert want < -1e-3  # the bias is not trivially zero here
    plain = evaluate(batch, p, nl)
    assert np.abs(r.forces - plain.forces).max() < 1e-10


def test_biased_forces_are_energy_gradients():
    batch, params, nl = _ens(n_structs=1)
    r = evaluate_udd(batch, params, nl, A, B)
    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(4):
        k, a = int(rng.integers(batch.n_atoms)), int(rng.integers(3))
        e = []
        for sgn in (1, -1):
            b2 = dataclasses.replace(batch, pos=batch.pos.astype(np.float64).copy())
            b2.pos[k, a] += sgn * h
            rr = evaluate_udd(b2, params, nl, A, B)
            e.append(rr.energy.mean(1).sum() + rr.bias_energy.sum())
        fd = -(e[0] - e[1]) / (2 * h)
        assert abs(fd - r.forces[k, a]) < 1e-6 * max(1.0, abs(fd))


def test_force_is_weighted_sum_of_head_forces():
    batch, params, nl = _ens(n_structs=1)
    r = evaluate_udd(batch, params, nl, A, B)
    M = params.spec.n_heads
    Fm = []
    for m in range(M):
        q = copy.deepcopy(params)
        q.W3 = params.W3[:, m:m + 1]
        q.b3 = params.b3[m:m + 1]
        q.spec = type(params.spec)(**{**params.spec.__dict__, "n_heads": 1})
        Fm.append(evaluate(batch, q, nl).forces)
    Fm = np.stack(Fm)
    E = r.energy[0]
    n = batch.n_atoms
    var = E.var()
    scale = 1.0 / (M * n * B * B)
    c = 1.0 / M - A * scale * math.exp(-var * scale) * 2.0 * (E - E.mean()) / M
    assert np.abs(np.tensordot(c, Fm, 1) - r.forces).max() < 1e-10
    assert np.abs(c - 1.0 / M).max() > 1e-6  # the weights differ from the plain mean


def test_zero_strength_is_unbiased():
    batch, params, nl = _ens()
    r = evaluate_udd(batch, params, nl, 0.0, B)
    plain = evaluate(batch, params, nl)
    assert np.all(r.bias_energy == 0.0)
    assert np.abs(r.forces - plain.forces).max() < 1e-12
    assert np.abs(r.stress - plain.stress).max() < 1e-12
