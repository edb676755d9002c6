"""Evaluations replayed from a HIP graph (gmnn_energy_forces_graph_create)
against eager evaluations of the same buffers: bitwise equal on every
replay, with eager work in between, and after the positions are rewritten in
place (the graph reads the buffers when it runs)."""
import numpy as np
import pytest
import torch

from workloads import make_workload
from gpu_helpers import gpu, need_gpu

pytestmark = gpu


def _snap(out):
    return [t.detach().cpu().numpy().copy() for t in (out.energy, out.forces, out.stress, out.atomic_energy)]


@pytest.mark.parametrize("plan", [None, (2, 16, 2)])
def test_graph_replays_equal_eager(plan):
    g = need_gpu()
    batch, params, spec = make_workload("liquid", n=400)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.model.r_cut, 0.5)  # skin: the list stays valid for small moves
    model = g.Model.from_params(params, "cuda")
    print(f"graph replay plan={plan}", flush=True)
    eager = g.EnergyForces(model, system, nl, precision="bf16", stress=True, plan=plan)
    ref = _snap(eager(sync=True))
    ev = g.EnergyForces(model, system, nl, precision="bf16", stress=True, plan=plan).capture(3)
    for rep in range(3):
        out = ev.replay(1)
        torch.cuda.synchronize()
        for a, b in zip(_snap(out), ref):
            assert np.array_equal(a, b), rep
        eager(sync=True)  # eager work between replays
    # new positions, same buffers: the replay sees them
    rng = np.random.default_rng(5)
    system.pos += torch.as_tensor(rng.normal(scale=0.02, size=tuple(system.pos.shape)).astype(np.float32),
                                  device="cuda")
    torch.cuda.synchronize()
    ref2 = _snap(eager(sync=True))
    assert not np.array_equal(ref2[1], ref[1])
    out = ev.replay(2)
    torch.cuda.synchronize()
    for a, b in zip(_snap(out), ref2):
        assert np.array_equal(a, b)
    ev.release()
