"""Uncertainty-driven bias (Section 2.3, eq. udd) on the GPU against the FP64
oracle: bias energies, biased forces and stress, unbiased head energies, in
both readouts and with the per-head force variance switched on (the
dump-interval mode of Section 3.5)."""
import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors, evaluate, evaluate_udd
from workloads import make_workload
from gpu_helpers import gpu, need_gpu

pytestmark = gpu

A, B = 1.0, 1.2
# split schedule with the tile readout, then the streamed one
PLANS = [None, (2, 32, 2)]


def _setup(g, n_structs=4):
    batch, params, spec = make_workload("ensemble", n_structs=n_structs)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.model.r_cut)
    model = g.Model.from_params(params, "cuda")
    return batch, params, spec, system, nl, model


@pytest.mark.parametrize("plan", PLANS)
@pytest.mark.parametrize("force_var", [False, True])
def test_udd_fp32_matches_oracle(plan, force_var):
    if force_var and plan is not None:
        pytest.skip("per-head backwards (force variance) run in the tile readout only")
    g = need_gpu()
    batch, params, spec, system, nl, model = _setup(g)
    ev = g.EnergyForces(model, system, nl, precision="fp32", stress=True, force_var=force_var, plan=plan,
                        udd=(A, B))
    out = ev(sync=True)
    onl = brute_force_neighbors(batch, spec.model.r_cut)
    ref = evaluate_udd(batch, params, onl, A, B)
    N = batch.n_atoms
    nb = np.diff(batch.atom_ptr)
    dEb = np.abs(out.bias_energy.cpu().numpy() - ref.bias_energy)
    dE = np.abs(out.energy.cpu().numpy() - ref.energy) / nb[:, None]
    dF = np.abs(out.forces.cpu().numpy()[:N] - ref.forces)
    dS = np.abs(out.stress.cpu().numpy() - ref.stress)
    print(f"udd plan {plan} var {force_var}: |dE_bias| {dEb.max():.2e}, |dE|/N {dE.max():.2e}, "
          f"max|dF| {dF.max():.2e}, max|dS| {dS.max():.2e}; bias {ref.bias_energy}")
    assert np.abs(ref.bias_energy).min() > 1e-4  # the bias acts
    assert dEb.max() < 1e-5 and dE.max() < 1e-5 and dF.max() < 1e-4 and dS.max() < 1e-6
    if force_var:
        unb = evaluate(batch, params, onl, want_force_var=True)
        assert np.allclose(out.force_var.cpu().numpy()[:N], unb.force_var, rtol=1e-3, atol=1e-5)
    # the bias changes the forces: the plain evaluation differs
    plain = g.EnergyForces(model, system, nl, precision="fp32", plan=plan)(sync=True)
    assert np.abs(plain.forces.cpu().numpy()[:N] - out.forces.cpu().numpy()[:N]).max() > 1e-3


def test_udd_bf16_within_budget():
    g = need_gpu()
    batch, params, spec, system, nl, model = _setup(g)
    out = g.EnergyForces(model, system, nl, precision="bf16", udd=(A, B))(sync=True)
    ref = evaluate_udd(batch, params, brute_force_neighbors(batch, spec.model.r_cut), A, B)
    F = out.forces.cpu().numpy()[: batch.n_atoms]
    rms = np.sqrt((ref.forces ** 2).mean())
    assert np.sqrt(((F - ref.forces) ** 2).mean()) < 1e-2 * rms
    assert np.abs(out.bias_energy.cpu().numpy() - ref.bias_energy).max() < 1e-3


def test_udd_rejects_fused_plan_and_single_head():
    g = need_gpu()
    from paper_2505_22168_amd import _capi as Acap
    batch, params, spec, system, nl, model = _setup(g, n_structs=2)
    with pytest.raises(Acap.GMNNError) as e:
        g.EnergyForces(model, system, nl, precision="fp32", plan=(1, 64), udd=(A, B))()
    assert e.value.status == Acap.GMNN_ERR_UNSUPPORTED
    b1, p1, s1 = make_workload("tiny")
    sys1 = g.System.from_batch(b1, "cuda")
    nl1 = g.build_neighbors(sys1, 5.0)
    m1 = g.Model.from_params(p1, "cuda")
    with pytest.raises(Acap.GMNNError) as e:
        g.EnergyForces(m1, sys1, nl1, precision="fp32", udd=(A, B))()
    assert e.value.status == Acap.GMNN_ERR_INVALID_ARG
