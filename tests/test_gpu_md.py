"""Device MD (velocity Verlet, skin list, HIP graph) vs the oracle
integrator; graph replay == eager launches bit for bit; time reversibility;
list rebuilds inside the graph."""
import numpy as np
import pytest
import torch

from oracle.md import velocity_verlet
from workloads import make_workload
from gpu_helpers import gpu, need_gpu

pytestmark = gpu

MASSES = {0: 6.94, 1: 30.974, 2: 15.999}   # Li, P, O stand-ins for the 3:1:4 lattice


def _setup(g, reps=(7, 7, 6), T=600.0, precision="fp32", skin=1.0):
    batch, params, spec = make_workload("solid", reps=reps)
    masses = np.array([MASSES[int(z)] for z in batch.species])
    v0 = g.maxwell_boltzmann(masses, T, seed=3)
    system = g.System.from_batch(batch, "cuda")
    model = g.Model.from_params(params, "cuda")
    md = g.MD(model, system, masses, dt=0.5, skin=skin, velocities=v0, precision=precision)
    return batch, params, masses, v0, system, md


def test_first_steps_match_oracle_integrator():
    g = need_gpu()
    batch, params, masses, v0, system, md = _setup(g, reps=(5, 5, 4))
    md.steps(10)
    torch.cuda.synchronize()
    assert md.status() == 0
    xs, vs, es = velocity_verlet(batch, params, batch.pos.astype(np.float64), v0.astype(np.float64), masses, 0.5, 10)
    x = system.pos.cpu().numpy().astype(np.float64)
    v = md.vel[: batch.n_atoms].cpu().numpy().astype(np.float64)
    assert np.abs(x - xs[-1]).max() < 2e-5
    assert np.abs(v - vs[-1]).max() < 2e-5
    assert abs(md.energy.cpu().numpy()[0, 0] - es[-1]) / batch.n_atoms < 2e-5


def test_graph_replay_equals_eager_bitwise():
    g = need_gpu()
    _, _, _, _, sys_a, md_a = _setup(g)
    md_a.steps(20)
    torch.cuda.synchronize()
    _, _, _, _, sys_b, md_b = _setup(g)
    md_b.capture(10)
    md_b.run(2)
    torch.cuda.synchronize()
    assert torch.equal(sys_a.pos, sys_b.pos)
    assert torch.equal(md_a.vel, md_b.vel)
    assert torch.equal(md_a.forces, md_b.forces)
    assert torch.equal(md_a.energy, md_b.energy)


def test_time_reversible():
    g = need_gpu()
    batch, params, masses, v0, system, md = _setup(g)
    x0 = system.pos.clone()
    md.capture(25)
    md.run(1)
    torch.cuda.synchronize()
    md.vel.neg_()
    md.run(1)
    torch.cuda.synchronize()
    assert (system.pos - x0).abs().max().item() < 2e-4
    assert (md.vel[: batch.n_atoms] + torch.as_tensor(v0, device="cuda")).abs().max().item() < 2e-4


def test_rebuilds_inside_graph_keep_forces_exact():
    """Hot start and a small skin: the list must be rebuilt several times in
    the graph; forces after 60 steps equal those of a fresh list."""
    g = need_gpu()
    batch, params, masses, v0, system, md = _setup(g, T=3000.0, skin=0.3)
    ref0 = md.ref_pos.clone()
    md.capture(30)
    md.run(2)
    torch.cuda.synchronize()
    assert md.status() == 0
    assert not torch.equal(md.ref_pos, ref0)          # at least one rebuild happened
    fresh = g.build_neighbors(system, 6.0, 0.0)
    out = g.energy_forces(md.model, system, fresh, precision="fp32", stress=False)
    torch.cuda.synchronize()
    # same forces up to FP32 summation order (the skin list orders lanes differently)
    assert (out.forces[: batch.n_atoms] - md.forces[: batch.n_atoms]).abs().max().item() < 1e-4
    disp = (system.pos - md.ref_pos)[: batch.n_atoms].norm(dim=1).max().item()
    assert disp <= 0.15 + 1e-6


def _setup_heads(g, n_heads=4, udd=None, var_every=0, reps=(5, 5, 4), precision="fp32"):
    """The lattice with a shallow ensemble of n_heads output heads."""
    import dataclasses
    from workloads.configs import make_params
    batch, params, spec = make_workload("solid", reps=reps)
    params = make_params(dataclasses.replace(spec.model, n_heads=n_heads, hidden=(64, 64)), 31)
    masses = np.array([MASSES[int(z)] for z in batch.species])
    v0 = g.maxwell_boltzmann(masses, 600.0, seed=3)
    system = g.System.from_batch(batch, "cuda")
    model = g.Model.from_params(params, "cuda")
    md = g.MD(model, system, masses, dt=0.5, skin=1.0, velocities=v0, precision=precision, udd=udd,
              var_every=var_every)
    return batch, params, masses, v0, system, md


def test_udd_biased_steps_match_oracle_integrator():
    """Uncertainty-driven dynamics (Section 2.3, eq. udd): the first steps
    against the oracle integrator on the biased potential, in a graph."""
    g = need_gpu()
    udd = (10.0, 2.0)
    batch, params, masses, v0, system, md = _setup_heads(g, udd=udd)
    md.capture(5)
    md.run(2)
    torch.cuda.synchronize()
    assert md.status() == 0
    xs, vs, es = velocity_verlet(batch, params, batch.pos.astype(np.float64), v0.astype(np.float64), masses, 0.5, 10,
                                 udd=udd)
    xu, vu, _ = velocity_verlet(batch, params, batch.pos.astype(np.float64), v0.astype(np.float64), masses, 0.5, 10)
    x = system.pos.cpu().numpy().astype(np.float64)
    v = md.vel[: batch.n_atoms].cpu().numpy().astype(np.float64)
    print(f"udd md: max|dv| vs biased oracle {np.abs(v - vs[-1]).max():.2e}, bias effect {np.abs(vs[-1] - vu[-1]).max():.2e}")
    assert np.abs(vs[-1] - vu[-1]).max() > 1e-4     # the bias moves the trajectory
    assert np.abs(x - xs[-1]).max() < 2e-5
    assert np.abs(v - vs[-1]).max() < 2e-5
    assert float(md.bias_energy.abs().sum().item()) > 0.0


def test_force_variance_every_nth_step_of_a_graph():
    """Mode switching (Section 3.5): the per-head force variance on every
    fifth step only; the trajectory equals the one without it (the mean of
    the head forces is the head-mean force, up to FP32 summation order), and
    the variance written on the graph's last step is that of the final
    positions."""
    g = need_gpu()
    _, _, _, _, sys_a, md_a = _setup_heads(g, var_every=5)
    md_a.capture(10)
    md_a.run(1)
    _, _, _, _, sys_b, md_b = _setup_heads(g)
    md_b.capture(10)
    md_b.run(1)
    torch.cuda.synchronize()
    assert (sys_a.pos - sys_b.pos).abs().max().item() < 1e-5
    assert (md_a.vel - md_b.vel).abs().max().item() < 1e-5
    nl = g.build_neighbors(sys_a, md_a.model.spec.r_cut, 0.0)
    ref = g.energy_forces(md_a.model, sys_a, nl, precision="fp32", force_var=True)
    torch.cuda.synchronize()
    n = sys_a.n_atoms
    assert float(md_a.force_var[:n].abs().max().item()) > 0.0
    assert torch.allclose(md_a.force_var[:n], ref.force_var[:n], rtol=1e-3, atol=1e-6)
    assert float(md_b.force_var.abs().max().item()) == 0.0   # never requested there
