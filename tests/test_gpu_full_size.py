"""Parity at full size and in narrow cells.

* The 100,000-atom solid-like lattice (r_c 6 A, 1 A skin) in the launch
  configuration the benchmark times (built-in plan): sampled rows of the
  11M-pair list bit-exact against the brute force, and energies and forces of
  sampled atoms against the FP64 oracle, which evaluates a non-periodic cluster
  cut around each sample (an atom's energy depends on atoms within r_c, its
  force on atoms within 2 r_c: cluster atoms that deep inside carry their
  periodic values).
* Cells narrower than the cutoff (Section 3.5: several images of one
  neighbour, and images of an atom itself, lie inside r_c): list bit-exact,
  FP32 energies/forces/stress against the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors, evaluate
from workloads import cluster_cut, make_batch, make_workload
from gpu_helpers import gpu, need_gpu, gpu_list_triples, oracle_triples

pytestmark = gpu


@pytest.fixture(scope="module")
def solid_full():
    g = need_gpu()
    batch, params, spec = make_workload("solid")
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.model.r_cut, spec.skin)
    model = g.Model.from_params(params, "cuda")
    return g, batch, params, spec, system, nl, model


def test_solid_full_list_sampled_rows(solid_full):
    g, batch, params, spec, system, nl, model = solid_full
    print(f"solid list: {batch.n_atoms} atoms, {nl.n_pairs} pairs", flush=True)
    assert nl.status == 0
    rows = np.arange(0, batch.n_atoms, 2503)
    ref = brute_force_neighbors(batch, spec.model.r_cut + spec.skin, rows=rows)
    t = gpu_list_triples(nl)
    got = t[np.isin(t[:, 0], rows)]
    assert np.array_equal(got, oracle_triples(ref))
    # the reverse index on the sampled rows' pairs
    rev = nl.rev[:nl.n_pairs].cpu().numpy().astype(np.int64)
    sel = np.nonzero(np.isin(t[:, 0], rows))[0]
    assert np.array_equal(t[rev[sel], 0], t[sel, 1]) and np.array_equal(t[rev[sel], 2:], -t[sel, 2:])


@pytest.mark.parametrize("plan", ["builtin", "auto"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_solid_full_sampled_parity(solid_full, precision, plan, tmp_path, monkeypatch):
    """Built-in plan and the autotuned one (the benchmark's default)."""
    g, batch, params, spec, system, nl, model = solid_full
    rc = spec.model.r_cut
    monkeypatch.setenv("GMNN_TUNE_CACHE", str(tmp_path / "tune.json"))
    ev = g.EnergyForces(model, system, nl, precision=precision, stress=True, plan=None if plan == "builtin" else "auto")
    if plan == "builtin":
        assert ev.plan == {"schedule": 2, "lanes_per_atom": 16, "readout": 2, "tile_atoms": 0}
    print(f"solid {precision} plan {ev.plan}", flush=True)
    out = ev(sync=True)
    F = out.forces.cpu().numpy()[: batch.n_atoms].astype(np.float64)
    Ei = out.atomic_energy.cpu().numpy()[: batch.n_atoms, 0].astype(np.float64)
    E = out.energy.cpu().numpy()[0, 0]
    assert abs(E - Ei.sum()) < 1e-9 * abs(E)
    R = 2 * rc + 3.0
    dF, dE, Fref = [], [], []
    for center in (0, 31337, 77777):
        cut, idx, dist = cluster_cut(batch, center, R)
        ref = evaluate(cut, params, brute_force_neighbors(cut, rc), want_stress=False)
        fi, ei = dist < R - 2 * rc, dist < R - rc
        dF.append(F[idx[fi]] - ref.forces[fi])
        Fref.append(ref.forces[fi])
        dE.append(Ei[idx[ei]] - ref.atomic[ei, 0])
    dF, dE, Fref = np.concatenate(dF), np.concatenate(dE), np.concatenate(Fref)
    rms = np.sqrt((Fref ** 2).mean())
    print(f"solid {precision}: {len(dF)} forces, {len(dE)} energies; max|dF| {np.abs(dF).max():.2e} eV/A "
          f"(RMS|F| {rms:.2f}), force RMSE {np.sqrt((dF ** 2).mean()):.2e}, max|dE_i| {np.abs(dE).max():.2e} eV",
          flush=True)
    assert len(dF) >= 20
    if precision == "fp32":
        assert np.abs(dF).max() < 1e-4
        assert np.abs(dE).max() < 1e-4
    else:
        # the BF16 budget: force RMSE <= 1% of RMS|F|, energies <= 1e-3 eV/atom
        assert np.sqrt((dF ** 2).mean()) < 1e-2 * rms
        assert np.abs(dE).max() < 1e-3


NARROW = [
    # one atom in a cubic cell narrower than r_c: only self images
    (np.zeros((1, 3), np.float32), np.zeros(1, np.int32), np.eye(3) * 3.1, 5.0),
    # three atoms of two species in a 4 A triclinic cell
    (np.array([[0.2, 0.3, 0.1], [1.9, 1.4, 0.8], [3.1, 2.7, 2.2]], np.float32), np.array([0, 1, 1], np.int32),
     np.array([[4.0, 0.0, 0.0], [0.9, 3.8, 0.0], [0.4, 0.6, 4.2]]), 5.0),
]


@pytest.mark.parametrize("case", range(len(NARROW)))
def test_cells_narrower_than_cutoff(case):
    g = need_gpu()
    pos, sp, cell, rc = NARROW[case]
    batch = make_batch([(pos, sp, cell, (1, 1, 1))])
    _, params, _ = make_workload("tiny")
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, rc)
    ref_nl = brute_force_neighbors(batch, rc)
    assert ref_nl.n_pairs > 0 and np.any(ref_nl.i == ref_nl.j)  # self images are listed
    assert np.array_equal(gpu_list_triples(nl), oracle_triples(ref_nl))
    model = g.Model.from_params(params, "cuda")
    out = g.energy_forces(model, system, nl, precision="fp32", stress=True)
    torch.cuda.synchronize()
    ref = evaluate(batch, params, ref_nl)
    n = batch.n_atoms
    assert abs(out.energy.cpu().numpy()[0, 0] - ref.energy[0, 0]) / n < 1e-5
    assert np.abs(out.forces.cpu().numpy()[:n] - ref.forces).max() < 1e-4
    assert np.abs(out.stress.cpu().numpy() - ref.stress).max() < 1e-6
