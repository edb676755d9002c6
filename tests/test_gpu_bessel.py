"""The Bessel-like radial basis (Section 2.1 names it beside the Gaussians)
on the GPU: energies, forces and stress against the FP64 oracle in every
schedule, the BF16 network within its budget, and training gradients."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors, evaluate, loss_and_param_grads
from oracle.gmnn import PARAM_NAMES
from workloads import make_workload
from workloads.configs import make_params
from gpu_helpers import gpu, need_gpu

pytestmark = gpu


def _bessel(name, hidden=None, seed=21, **kw):
    batch, params, spec = make_workload(name, **kw)
    s2 = dataclasses.replace(spec.model, basis="bessel", hidden=hidden or spec.model.hidden)
    return batch, make_params(s2, seed), s2


# (schedule, lanes per atom, readout): fused, split with the tile readout,
# split with the streamed readout
PLANS = [None, (2, 16, 1), (2, 32, 2)]


@pytest.mark.parametrize("plan", PLANS)
@pytest.mark.parametrize("name,kw", [("tiny", {}), ("liquid", dict(n=400, sweeps=2)),
                                     ("train", dict(n_structs=2, n_lo=100, n_hi=160))])
def test_bessel_fp32_matches_oracle(name, kw, plan):
    g = need_gpu()
    batch, params, spec = _bessel(name, **kw)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.r_cut)
    model = g.Model.from_params(params, "cuda")
    out = g.EnergyForces(model, system, nl, precision="fp32", stress=True, plan=plan)(sync=True)
    ref = evaluate(batch, params, brute_force_neighbors(batch, spec.r_cut))
    nb = np.diff(batch.atom_ptr)
    dE = np.abs(out.energy.cpu().numpy() - ref.energy) / nb[:, None]
    dF = np.abs(out.forces.cpu().numpy()[: batch.n_atoms] - ref.forces)
    dS = np.abs(out.stress.cpu().numpy() - ref.stress)
    print(f"bessel {name} plan {plan}: |dE|/N {dE.max():.2e}, max|dF| {dF.max():.2e}, max|dS| {dS.max():.2e}")
    assert dE.max() < 1e-5 and dF.max() < 1e-4 and dS.max() < 1e-6


def test_bessel_bf16_within_budget():
    g = need_gpu()
    batch, params, spec = _bessel("train", n_structs=2, n_lo=100, n_hi=160)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.r_cut)
    model = g.Model.from_params(params, "cuda")
    out = g.EnergyForces(model, system, nl, precision="bf16", stress=True)(sync=True)
    onl = brute_force_neighbors(batch, spec.r_cut)
    ref16, ref64 = evaluate(batch, params, onl, bf16=True), evaluate(batch, params, onl)
    F = out.forces.cpu().numpy()[: batch.n_atoms]
    rms = np.sqrt((ref64.forces ** 2).mean())
    nb = np.diff(batch.atom_ptr)
    assert np.abs(F - ref16.forces).max() < 1e-2 * rms
    assert np.sqrt(((F - ref64.forces) ** 2).mean()) < 1e-2 * rms
    assert (np.abs(out.energy.cpu().numpy() - ref64.energy) / nb[:, None]).max() < 1e-3


def test_bessel_param_gradients_match_oracle():
    g = need_gpu()
    batch, params, spec = _bessel("train", hidden=(64, 64), n_structs=3, n_lo=30, n_hi=70)
    teacher = make_params(spec, 121)
    onl = brute_force_neighbors(batch, spec.r_cut)
    rt = evaluate(batch, teacher, onl)
    L, gref, dLdE, dLdF = loss_and_param_grads(batch, params, onl, rt.energy_mean, rt.forces)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.r_cut)
    model = g.Model.from_params(params, "cuda")
    grads = g.param_grads(model, system, nl, dLdE, dLdF)
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        got = grads[k].cpu().numpy().astype(np.float64).reshape(np.shape(gref[k]))
        err = np.linalg.norm(got - gref[k]) / max(np.linalg.norm(gref[k]), 1e-30)
        assert err < 1e-4, (k, err)


def test_bessel_position_gradients_match_oracle():
    """The Hessian-vector product of the positions' gradient with the
    Bessel-like basis (its second radial derivatives)."""
    g = need_gpu()
    batch, params, spec = _bessel("train", hidden=(64, 64), n_structs=3, n_lo=30, n_hi=70)
    teacher = make_params(spec, 121)
    onl = brute_force_neighbors(batch, spec.r_cut)
    rt = evaluate(batch, teacher, onl)
    L, gref, dLdE, dLdF, gx = loss_and_param_grads(batch, params, onl, rt.energy_mean, rt.forces, want_pos=True)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.r_cut)
    model = g.Model.from_params(params, "cuda")
    dpos = torch.empty((batch.n_atoms, 3), dtype=torch.float32, device="cuda")
    g.param_grads(model, system, nl, dLdE, dLdF, dL_dpos=dpos)
    torch.cuda.synchronize()
    got = dpos.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - gx) / np.linalg.norm(gx) < 1e-4
