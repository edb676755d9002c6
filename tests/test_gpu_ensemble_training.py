"""Shallow-ensemble training step on the GPU through the C ABI vs the FP64
oracle (Section 2.2, eq. nll; Section 3.4): per-head forces, the loss terms
and their per-head gradients, the per-head double backward, Adam with
parameter groups and a schedule, and the whole step."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors, evaluate
from oracle.ensemble_training import LossSpec as OracleLoss, adam_step, ensemble_loss_and_param_grads, \
    ensemble_loss_grads, lr_factor
from oracle.gmnn import PARAM_NAMES
from workloads import make_workload
from workloads.configs import make_params
from gpu_helpers import gpu, need_gpu

pytestmark = gpu

GROUP = {"beta": "embedding", "W1": "nn", "b1": "nn", "W2": "nn", "b2": "nn", "W3": "nn", "b3": "nn",
         "scale": "scale", "shift": "shift"}


def _case(hidden=(64, 64), heads=4, **kw):
    batch, params, spec = make_workload("train", **kw)
    s2 = dataclasses.replace(spec.model, hidden=hidden, n_heads=heads)
    params = make_params(s2, 17)
    teacher = make_params(dataclasses.replace(s2, n_heads=1), 117)
    onl = brute_force_neighbors(batch, s2.r_cut)
    rt = evaluate(batch, teacher, onl)
    return batch, params, onl, rt.energy_mean, rt.forces


def _setup(g, batch, params):
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, params.spec.r_cut)
    model = g.Model.from_params(params, "cuda")
    return system, nl, model


def _rel(got, ref):
    return np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)


def test_per_head_forces_match_oracle():
    g = need_gpu()
    batch, params, onl, Er, Fr = _case(n_structs=3, n_lo=30, n_hi=60)
    system, nl, model = _setup(g, batch, params)
    out = g.energy_forces(model, system, nl, precision="fp32", stress=False, force_var=True)
    torch.cuda.synchronize()
    ref = ensemble_loss_and_param_grads(batch, params, onl, Er, Fr, OracleLoss())
    Fh = out.forces_heads.cpu().numpy()[:, : batch.n_atoms]
    assert np.abs(Fh - ref.forces_heads).max() < 1e-4
    assert np.abs(out.energy.cpu().numpy() - ref.energy_heads).max() / batch.n_atoms < 1e-5
    # the head mean of the per-head forces is the force of the mean energy
    assert np.abs(Fh.mean(0) - out.forces.cpu().numpy()[: batch.n_atoms]).max() < 1e-5


@pytest.mark.parametrize("ekind,fkind,per_atom", [("crps", "crps", True), ("nll", "nll", False),
                                                  ("mse", "crps", True), ("nll", "mse", True)])
def test_loss_terms_and_head_gradients_match_oracle(ekind, fkind, per_atom):
    """Seeded per-head energies and forces (300 structures, 1000 atoms: several
    blocks and a ragged tail in both terms) through gmnn_ensemble_loss."""
    g = need_gpu()
    rng = np.random.default_rng(21)
    B, N, M = 300, 1000, 7
    ptr = np.concatenate([[0], np.sort(rng.choice(np.arange(1, N), B - 1, replace=False)), [N]]).astype(np.int64)
    nb = np.diff(ptr).astype(np.float64)
    E = (-4.0 * nb)[:, None] + rng.normal(size=(B, M)) * 0.05 * np.sqrt(nb)[:, None]
    Er = -4.0 * nb + rng.normal(size=B) * 0.05 * np.sqrt(nb)
    F = (rng.normal(size=(N, 3))[None] + 0.1 * rng.normal(size=(M, N, 3))).astype(np.float32)
    Fr = (rng.normal(size=(N, 3))).astype(np.float32)
    spec = g.LossSpec(ekind, fkind, w_energy=0.8, w_force=1.7, energy_per_atom=per_atom, var_floor=1e-6)
    ospec = OracleLoss(ekind, fkind, 0.8, 1.7, per_atom, 1e-6)
    pos = np.zeros((N, 3), np.float32)
    system = g.System(pos, np.zeros(N, np.int32), np.tile(np.eye(3) * 10.0, (B, 1, 1)), np.zeros((B, 3), np.uint8),
                      ptr, "cuda")
    loss, dE, dF = g.ensemble_loss(system, torch.tensor(E, device="cuda"), torch.tensor(F, device="cuda"), Er, Fr,
                                   spec)
    torch.cuda.synchronize()
    LE, LF, gE, gF = ensemble_loss_grads(E, F.astype(np.float64), Er, Fr.astype(np.float64), nb, ospec)
    loss = loss.cpu().numpy()
    assert abs(loss[0] - LE) <= 1e-12 * max(1.0, abs(LE)), (loss[0], LE)
    assert abs(loss[1] - LF) <= 1e-12 * max(1.0, abs(LF)), (loss[1], LF)
    assert np.abs(dE.cpu().numpy() - gE).max() <= 1e-11 * np.abs(gE).max()
    dFg = dF.cpu().numpy().astype(np.float64)
    assert np.abs(dFg - gF).max() <= 1e-6 * np.abs(gF).max()


def test_per_head_backward_matches_oracle():
    """The oracle's upstream gradients dL/dE^m, dL/dF^m (CRPS terms) into
    gmnn_backward with GMNN_BACKWARD_PER_HEAD: every parameter gradient
    against the oracle's (relative l2 < 1e-4, FP32)."""
    g = need_gpu()
    batch, params, onl, Er, Fr = _case(n_structs=3, n_lo=30, n_hi=60)
    ref = ensemble_loss_and_param_grads(batch, params, onl, Er, Fr, OracleLoss(var_floor=1e-6))
    system, nl, model = _setup(g, batch, params)
    grads = g.param_grads(model, system, nl, ref.dL_dE, ref.dL_dF, per_head=True)
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        got = grads[k].cpu().numpy().astype(np.float64).reshape(np.shape(ref.grads[k]))
        err = _rel(got, ref.grads[k])
        print(k, err)
        assert err < 1e-4, (k, err)


def test_per_head_backward_bf16_within_budget():
    g = need_gpu()
    batch, params, onl, Er, Fr = _case(hidden=(128, 128), n_structs=2, n_lo=40, n_hi=60)
    ref = ensemble_loss_and_param_grads(batch, params, onl, Er, Fr, OracleLoss("nll", "crps", var_floor=1e-6))
    system, nl, model = _setup(g, batch, params)
    grads = g.param_grads(model, system, nl, ref.dL_dE, ref.dL_dF, per_head=True, precision="bf16")
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        err = _rel(grads[k].cpu().numpy().astype(np.float64).reshape(np.shape(ref.grads[k])), ref.grads[k])
        assert err < 3e-2, (k, err)


def test_one_head_per_head_backward_equals_head_mean_backward():
    """With one head the per-head backward is the head-mean backward, bitwise."""
    g = need_gpu()
    batch, params, onl, Er, Fr = _case(heads=1, n_structs=2, n_lo=30, n_hi=50)
    system, nl, model = _setup(g, batch, params)
    rng = np.random.default_rng(3)
    dE = rng.normal(size=(batch.n_structs, 1))
    dF = rng.normal(size=(1, batch.n_atoms, 3)).astype(np.float32)
    a = g.param_grads(model, system, nl, dE, dF, per_head=True)
    b = g.param_grads(model, system, nl, dE[:, 0], dF[0])
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        assert torch.equal(a[k], b[k]), k


def test_adam_with_groups_and_schedule_matches_oracle():
    """Three Adam steps with seeded gradients, a frozen embedding group and a
    cyclic cosine schedule against the oracle's FP64 Adam from the same FP32
    start; then the re-packed weights evaluate as a freshly built model."""
    g = need_gpu()
    batch, params, onl, Er, Fr = _case(n_structs=2, n_lo=20, n_hi=30)
    system, nl, model = _setup(g, batch, params)
    lr = {"embedding": 0.0, "nn": 2e-3, "scale": 1e-2, "shift": 5e-3}
    sched = dict(kind="cosine", period=4, decay_factor=0.9)
    opt = g.Adam(model, lr, schedule=sched)
    p = {k: model.tensors[k].cpu().numpy().astype(np.float64) for k in PARAM_NAMES}
    start = {k: v.copy() for k, v in p.items()}
    m1 = {k: np.zeros_like(v) for k, v in p.items()}
    m2 = {k: np.zeros_like(v) for k, v in p.items()}
    rng = np.random.default_rng(8)
    for t in range(1, 4):
        gr = {k: (rng.normal(size=p[k].shape) * 10.0 ** rng.uniform(-3, 0)).astype(np.float32) for k in PARAM_NAMES}
        opt.step({k: torch.tensor(v, device="cuda") for k, v in gr.items()})
        f = lr_factor("cosine", t - 1, period=4, decay_factor=0.9)
        p, m1, m2 = adam_step(p, {k: v.astype(np.float64) for k, v in gr.items()}, m1, m2, t,
                              {k: v * f for k, v in lr.items()})
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        got = model.tensors[k].cpu().numpy().astype(np.float64)
        tol = 1e-5 * max(lr[GROUP[k]], 1e-12) + 2e-7 * np.abs(p[k])
        assert np.all(np.abs(got - p[k]) <= tol), (k, np.abs(got - p[k]).max())
    assert np.array_equal(model.tensors["beta"].cpu().numpy().astype(np.float64), start["beta"])
    fresh = g.Model(params.spec, {k: model.tensors[k].cpu().numpy() for k in PARAM_NAMES}, "cuda")
    a = g.energy_forces(model, system, nl, precision="fp32", stress=False)
    b = g.energy_forces(fresh, system, nl, precision="fp32", stress=False)
    torch.cuda.synchronize()
    assert torch.equal(a.energy, b.energy) and torch.equal(a.forces, b.forces)


@pytest.mark.parametrize("kind", ["crps", "nll"])
def test_training_step_matches_oracle(kind):
    """EnsembleTrainer.step (per-head forces -> loss -> per-head backward ->
    Adam) against the oracle's loss, gradient and Adam update.  The first
    Adam step moves every entry by about its learning rate along -sign(g),
    so entries whose oracle gradient is within FP32 noise of zero may move
    either way; the others must match the oracle's update."""
    g = need_gpu()
    batch, params, onl, Er, Fr = _case(n_structs=3, n_lo=30, n_hi=50)
    spec = OracleLoss(kind, kind, w_energy=1.0, w_force=1.0, energy_per_atom=True, var_floor=1e-6)
    ref = ensemble_loss_and_param_grads(batch, params, onl, Er, Fr, spec)
    system, nl, model = _setup(g, batch, params)
    lr = {"embedding": 1e-3, "nn": 1e-3, "scale": 1e-3, "shift": 1e-3}
    opt = g.Adam(model, lr)
    start = {k: model.tensors[k].cpu().numpy().astype(np.float64) for k in PARAM_NAMES}
    tr = g.EnsembleTrainer(model, system, nl, Er, Fr, g.LossSpec(kind, kind, 1.0, 1.0, True, 1e-6), opt)
    loss = tr.step().cpu().numpy()
    torch.cuda.synchronize()
    assert abs(loss[0] - ref.loss_energy) < 1e-5 * max(1.0, abs(ref.loss_energy))
    assert abs(loss[1] - ref.loss_force) < 1e-5 * max(1.0, abs(ref.loss_force))
    for k in PARAM_NAMES:
        got_g = tr.grads[k].cpu().numpy().astype(np.float64).reshape(np.shape(ref.grads[k]))
        assert _rel(got_g, ref.grads[k]) < 1e-4, k
        p, _, _ = adam_step({k: start[k].copy()}, {k: ref.grads[k]}, {k: np.zeros_like(start[k])},
                            {k: np.zeros_like(start[k])}, 1, lr)
        got = model.tensors[k].cpu().numpy().astype(np.float64)
        clear = np.abs(ref.grads[k]) > 1e-3 * np.abs(ref.grads[k]).max()
        assert np.all(np.abs(got - p[k])[clear] <= 1e-6 + 1e-6 * np.abs(p[k])[clear]), k
        assert np.all(np.abs(got - start[k]) <= 1.0001e-3 + 1e-6 * np.abs(start[k])), k


def test_per_head_position_gradients_match_oracle():
    """dL/dx of the ensemble loss: the positions' gradients of the per-head
    double backwards summed in head order, against the oracle's."""
    g = need_gpu()
    batch, params, onl, Er, Fr = _case(n_structs=3, n_lo=30, n_hi=60)
    ref = ensemble_loss_and_param_grads(batch, params, onl, Er, Fr, OracleLoss("crps", "nll", var_floor=1e-4))
    system, nl, model = _setup(g, batch, params)
    dpos = torch.empty((batch.n_atoms, 3), dtype=torch.float32, device="cuda")
    g.param_grads(model, system, nl, ref.dL_dE, ref.dL_dF, per_head=True, dL_dpos=dpos)
    torch.cuda.synchronize()
    got = dpos.cpu().numpy().astype(np.float64)
    assert _rel(got, ref.dL_dpos) < 1e-4, _rel(got, ref.dL_dpos)


@pytest.mark.parametrize("lanes16", [False, True])
def test_per_head_backward_multi_chunk(lanes16):
    """Above 600 atoms (several split-K chunks and species blocks per head)
    and with the 16-lane pair kernels: per-head parameter and position
    gradients against the oracle."""
    g = need_gpu()
    batch, params, onl, Er, Fr = _case(n_structs=2, n_lo=330, n_hi=400)
    assert batch.n_atoms > 600
    ref = ensemble_loss_and_param_grads(batch, params, onl, Er, Fr, OracleLoss("crps", "crps", var_floor=1e-6))
    system, nl, model = _setup(g, batch, params)
    dpos = torch.empty((batch.n_atoms, 3), dtype=torch.float32, device="cuda")
    grads = g.param_grads(model, system, nl, ref.dL_dE, ref.dL_dF, per_head=True, lanes16=lanes16, dL_dpos=dpos)
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        err = _rel(grads[k].cpu().numpy().astype(np.float64).reshape(np.shape(ref.grads[k])), ref.grads[k])
        assert err < 1e-4, (k, err)
    assert _rel(dpos.cpu().numpy().astype(np.float64), ref.dL_dpos) < 1e-4


def test_loss_with_an_empty_structure_matches_oracle():
    """A structure without atoms in the batch: no per-atom energy term, zero
    gradients for its heads, the other terms unchanged."""
    g = need_gpu()
    rng = np.random.default_rng(31)
    ptr = np.array([0, 5, 5, 12, 20], dtype=np.int64)
    B, N, M = 4, 20, 5
    nb = np.diff(ptr).astype(np.float64)
    E = (-3.0 * nb)[:, None] + rng.normal(size=(B, M)) * 0.1
    E[1] = 0.0
    Er = -3.0 * nb + rng.normal(size=B) * 0.1
    F = rng.normal(size=(M, N, 3)).astype(np.float32)
    Fr = rng.normal(size=(N, 3)).astype(np.float32)
    system = g.System(np.zeros((N, 3), np.float32), np.zeros(N, np.int32), np.tile(np.eye(3) * 10.0, (B, 1, 1)),
                      np.zeros((B, 3), np.uint8), ptr, "cuda")
    loss, dE, dF = g.ensemble_loss(system, torch.tensor(E, device="cuda"), torch.tensor(F, device="cuda"), Er, Fr,
                                   g.LossSpec("nll", "crps", 1.0, 1.0, True, 1e-4))
    torch.cuda.synchronize()
    LE, LF, gE, gF = ensemble_loss_grads(E, F.astype(np.float64), Er, Fr.astype(np.float64), nb,
                                         OracleLoss("nll", "crps", 1.0, 1.0, True, 1e-4))
    loss = loss.cpu().numpy()
    assert np.isfinite(loss).all()
    assert abs(loss[0] - LE) <= 1e-12 * max(1.0, abs(LE)) and abs(loss[1] - LF) <= 1e-12 * max(1.0, abs(LF))
    assert np.all(dE.cpu().numpy()[1] == 0.0)
    assert np.abs(dE.cpu().numpy() - gE).max() <= 1e-11 * np.abs(gE).max()
