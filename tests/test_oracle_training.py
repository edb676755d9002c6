"""Pins of the oracle training gradients (energy + force loss): directional
finite differences over all parameters, the closed form of dL/dmu, and the
upstream gradients dL/dE, dL/dF."""
import copy

import numpy as np
import pytest

from oracle import brute_force_neighbors, evaluate, loss_and_param_grads
from oracle.gmnn import PARAM_NAMES
from workloads import make_workload


@pytest.fixture(scope="module")
def setup():
    b, p, s = make_workload("train", n_structs=2, n_lo=20, n_hi=30)
    # small network for speed; labels from a teacher with another seed
    from workloads.configs import ModelSpec, make_params
    spec = ModelSpec(n_species=5, r_cut=5.0, hidden=(16, 16), psi_scale=s.model.psi_scale)
    p = make_params(spec, 7)
    t = make_params(spec, 107)
    nl = brute_force_neighbors(b, 5.0)
    rt = evaluate(b, t, nl)
    return b, p, nl, rt.energy_mean, rt.forces


def _loss(b, p, nl, Er, Fr):
    r = evaluate(b, p, nl)
    nb = np.diff(b.atom_ptr)
    return (((r.energy_mean - Er) / nb) ** 2).sum() / b.n_structs + ((r.forces - Fr) ** 2).sum() / (3 * b.n_atoms)


def test_loss_value_matches_definition(setup):
    b, p, nl, Er, Fr = setup
    L, _, _, _ = loss_and_param_grads(b, p, nl, Er, Fr)
    assert abs(L - _loss(b, p, nl, Er, Fr)) < 1e-12 * max(1, L)


def test_directional_derivatives(setup):
    b, p, nl, Er, Fr = setup
    L, g, _, _ = loss_and_param_grads(b, p, nl, Er, Fr)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(4):
        v = {k: rng.normal(size=np.shape(getattr(p, k))) for k in PARAM_NAMES}
        ana = sum(float((g[k] * v[k]).sum()) for k in PARAM_NAMES)
        vals = []
        for s in (1, -1):
            q = copy.deepcopy(p)
            for k in PARAM_NAMES:
                setattr(q, k, getattr(p, k) + s * h * v[k])
            vals.append(_loss(b, q, nl, Er, Fr))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - ana) < 1e-6 * max(1.0, abs(ana))


def test_shift_gradient_closed_form(setup):
    """Forces do not depend on mu; dL/dmu_z = 2/B sum_b ((E_b - E_ref_b)/N_b) n_{z,b}/N_b."""
    b, p, nl, Er, Fr = setup
    _, g, dLdE, dLdF = loss_and_param_grads(b, p, nl, Er, Fr)
    r = evaluate(b, p, nl)
    nb = np.diff(b.atom_ptr)
    want = np.zeros(p.spec.n_species)
    for bi in range(b.n_structs):
        sp = b.species[b.atom_ptr[bi]:b.atom_ptr[bi + 1]]
        cnt = np.bincount(sp, minlength=p.spec.n_species)
        want += 2.0 / b.n_structs * (r.energy_mean[bi] - Er[bi]) / nb[bi] * cnt / nb[bi]
    assert np.allclose(g["shift"], want, rtol=1e-10, atol=1e-14)
    assert np.allclose(dLdE, 2.0 / b.n_structs * (r.energy_mean - Er) / nb ** 2, rtol=1e-10)
    assert np.allclose(dLdF, 2.0 / (3 * b.n_atoms) * (r.forces - Fr), rtol=1e-10, atol=1e-16)


def test_position_gradient_directional_differences(setup):
    """dL/dx against five-point differences of the loss along random position
    displacements (list built with a skin so no pair leaves it), and zero net
    gradient (the loss is invariant under a rigid translation)."""
    import dataclasses
    b, p, _, Er, Fr = setup
    nl = brute_force_neighbors(b, 5.5)
    _, _, _, _, gx = loss_and_param_grads(b, p, nl, Er, Fr, want_pos=True)
    assert np.abs(gx.sum(0)).max() < 1e-10 * max(1.0, np.abs(gx).max())
    rng = np.random.default_rng(2)
    h = 1e-4
    for _ in range(2):
        v = rng.normal(size=b.pos.shape)
        ana = float((gx * v).sum())

        def L(t):
            bt = dataclasses.replace(b, pos=b.pos.astype(np.float64) + t * v)
            return _loss(bt, p, nl, Er, Fr)

        fd = (8 * (L(h) - L(-h)) - (L(2 * h) - L(-2 * h))) / (12 * h)
        assert abs(fd - ana) < 1e-6 * max(1.0, abs(ana)), (fd, ana)
