"""Degenerate inputs through the C ABI: an empty structure inside a batch,
an isolated atom (no neighbour: Psi = 0, zero force), a system of zero
atoms, and rows longer than the list build handles (flagged; the list stays
well formed)."""
import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors, evaluate
from workloads import make_batch, make_workload
from gpu_helpers import gpu, need_gpu

pytestmark = gpu


def _edge_batch():
    tiny, params, spec = make_workload("tiny")
    s0 = (tiny.pos, tiny.species, tiny.cell[0], tiny.pbc[0])
    empty = (np.zeros((0, 3), np.float32), np.zeros(0, np.int32), np.eye(3) * 9.0, (1, 1, 1))
    lone = (np.array([[3.0, 4.0, 5.0]], np.float32), np.array([1], np.int32), np.eye(3) * 30.0, (0, 0, 0))
    pair = (np.array([[1.0, 1.0, 1.0], [2.2, 1.3, 0.8]], np.float32), np.array([0, 1], np.int32),
            np.eye(3) * 12.0, (0, 1, 0))
    return make_batch([s0, empty, lone, pair]), params, spec


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("plan", [None, (2, 16, 1), (2, 32, 2)])
def test_empty_structure_isolated_atom_and_dimer(precision, plan):
    g = need_gpu()
    batch, params, spec = _edge_batch()
    print(f"edge batch {precision} plan={plan}", flush=True)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.model.r_cut)
    model = g.Model.from_params(params, "cuda")
    out = g.EnergyForces(model, system, nl, precision=precision, stress=True, plan=plan)(sync=True)
    ref = evaluate(batch, params, brute_force_neighbors(batch, spec.model.r_cut), bf16=(precision == "bf16"))
    E = out.energy.cpu().numpy()
    F = out.forces.cpu().numpy()[: batch.n_atoms]
    tol_e, tol_f = (1e-4, 1e-4) if precision == "fp32" else (2e-3, 2e-3)
    assert np.abs(E - ref.energy).max() < tol_e * max(1.0, np.abs(ref.energy).max())
    assert np.abs(F - ref.forces).max() < tol_f * max(1.0, np.abs(ref.forces).max())
    assert np.all(E[1] == 0.0)                       # the empty structure
    assert np.all(out.stress.cpu().numpy()[1] == 0.0)
    lone = int(batch.atom_ptr[2])
    assert np.all(F[lone] == 0.0)                    # no neighbour, no force
    assert np.abs(F[lone + 1] + F[lone + 2]).max() < 1e-5  # the dimer's forces cancel


def test_zero_atoms():
    g = need_gpu()
    empty = (np.zeros((0, 3), np.float32), np.zeros(0, np.int32), np.eye(3) * 9.0, (1, 1, 1))
    batch = make_batch([empty])
    _, params, spec = make_workload("tiny")
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.model.r_cut)
    assert nl.n_pairs == 0
    model = g.Model.from_params(params, "cuda")
    for plan in (None, (2, 16, 1), (2, 16, 2)):
        out = g.EnergyForces(model, system, nl, precision="fp32", stress=True, plan=plan)(sync=True)
        assert np.all(out.energy.cpu().numpy() == 0.0)


def test_row_too_long_flagged_list_well_formed():
    """1300 atoms packed into a 4.5 A open box: every row holds more than the
    1024 neighbours the build sorts; the flag is raised (GMNN_SYNC turns it
    into an error) and every index of the list stays inside the system."""
    g = need_gpu()
    from paper_2505_22168_amd import _capi as A
    rng = np.random.default_rng(11)
    n = 1300
    pos = rng.uniform(0.0, 4.5, size=(n, 3)).astype(np.float32)
    batch = make_batch([(pos, np.zeros(n, np.int32), np.eye(3) * 4.5, (0, 0, 0))])
    system = g.System.from_batch(batch, "cuda")
    import ctypes as C
    lib = A.load()
    sysc = system.c()
    nl = g.NeighborList(n, n * n, "cuda")  # room for every pair: the rows are filled
    # sentinels a well-formed list cannot hold (an image code with its top byte
    # set): every slot the list reports must be overwritten by the build
    nl.j.fill_(n - 1)
    nl.shift.fill_(0x7F000000)
    nbytes = lib.gmnn_neighbors_workspace_bytes(C.byref(sysc), 5.0, 0.0)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    nlc = nl.c()
    st = lib.gmnn_build_neighbors(C.byref(sysc), 5.0, 0.0, C.byref(nlc), 0, C.c_void_p(ws.data_ptr()), nbytes,
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == A.GMNN_OK
    torch.cuda.synchronize()
    assert nl.status & A.GMNN_FLAG_ROW_TOO_LONG
    nlc = nl.c()
    st = lib.gmnn_build_neighbors(C.byref(sysc), 5.0, 0.0, C.byref(nlc), A.GMNN_SYNC, C.c_void_p(ws.data_ptr()),
                                  nbytes, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == A.GMNN_ERR_DEVICE_FLAG
    P = nl.n_pairs
    j = nl.j[:P].cpu().numpy()
    rev = nl.rev[:P].cpu().numpy()
    assert j.min() >= 0 and j.max() < n
    assert rev.min() >= 0 and rev.max() < P
    # truncated rows reserve exactly the slots they fill
    lengths = np.diff(nl.row_ptr.cpu().numpy())
    assert lengths.max() == 1024 and lengths.sum() == P
    sh = nl.shift[:P].cpu().numpy()
    assert not np.any(sh == 0x7F000000)


def test_output_status_word_flags_zero_distance_and_nonfinite():
    """A listed pair moved to zero distance, and a non-finite position, after
    the list was built: the evaluation leaves the pair out and raises the
    output status bits; GMNN_SYNC turns them into GMNN_ERR_DEVICE_FLAG."""
    g = need_gpu()
    from paper_2505_22168_amd import _capi as A
    batch, params, spec = make_workload("tiny")
    model = g.Model.from_params(params, "cuda")
    for what in ("coincident", "nonfinite"):
        system = g.System.from_batch(batch, "cuda")
        nl = g.build_neighbors(system, spec.model.r_cut, 0.5)
        ev = g.EnergyForces(model, system, nl, precision="fp32")
        ev(sync=True)
        assert int(ev.out.status.item()) == 0
        if what == "coincident":
            n = nl.n_pairs
            rows = nl.rows()[:n].cpu().numpy()
            same = np.nonzero((rows == 0) & (nl.shift[:n].cpu().numpy() == 0))[0]
            j = int(nl.j[int(same[0])].item())  # a neighbour of atom 0 in the same image
            system.pos[j] = system.pos[0]
            flag = A.GMNN_FLAG_COINCIDENT
        else:
            system.pos[5, 1] = float("nan")
            flag = A.GMNN_FLAG_NONFINITE
        ev()
        torch.cuda.synchronize()
        assert int(ev.out.status.item()) & flag
        with pytest.raises(A.GMNNError) as e:
            ev(sync=True)
        assert e.value.status == A.GMNN_ERR_DEVICE_FLAG


def test_energy_mean_over_heads_from_the_library():
    g = need_gpu()
    batch, params, spec = make_workload("ensemble", n_structs=5)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, 5.0)
    model = g.Model.from_params(params, "cuda")
    out = g.EnergyForces(model, system, nl, precision="fp32")(sync=True)
    E = out.energy.cpu().numpy()
    assert np.allclose(out.energy_mean.cpu().numpy(), E.mean(1), rtol=1e-15, atol=0)
