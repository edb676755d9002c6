"""GPU neighbour list vs the oracle brute force: bit-exact after canonical
sorting (the device list is canonical by construction), reverse index,
capacity and status handling."""
import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors
from workloads import make_batch, make_workload
from gpu_helpers import gpu, need_gpu, gpu_list_triples, oracle_triples

pytestmark = gpu


def _check_rev(nl):
    n = nl.n_pairs
    rev = nl.rev[:n].cpu().numpy().astype(np.int64)
    t = gpu_list_triples(nl)
    assert np.array_equal(rev[rev], np.arange(n))                 # involution
    assert np.array_equal(t[rev, 0], t[:, 1]) and np.array_equal(t[rev, 1], t[:, 0])
    assert np.array_equal(t[rev, 2:], -t[:, 2:])


def _build(g, batch, rc, skin=0.0, **kw):
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, rc, skin, **kw)
    return system, nl


@pytest.mark.parametrize("name,kw", [("tiny", {}), ("ensemble", dict(n_structs=6)),
                                     ("train", dict(n_structs=3, n_lo=100, n_hi=200))])
def test_list_bit_exact(name, kw):
    g = need_gpu()
    batch, params, spec = make_workload(name, **kw)
    _, nl = _build(g, batch, spec.model.r_cut)
    ref = brute_force_neighbors(batch, spec.model.r_cut)
    assert nl.status == 0
    assert nl.n_pairs == ref.n_pairs
    assert np.array_equal(gpu_list_triples(nl), oracle_triples(ref))
    _check_rev(nl)


def test_list_triclinic_and_mixed_pbc():
    g = need_gpu()
    rng = np.random.default_rng(11)
    structs = []
    for k in range(5):
        n = int(rng.integers(3, 40))
        cell = np.array([[6.0 + k, 0, 0], [1.7, 5.5, 0], [-1.1, 0.8, 7.0]])
        frac = rng.random((n, 3)) * 1.8 - 0.4                    # atoms outside the cell too
        pos = (frac @ cell).astype(np.float32)
        pbc = [(1, 1, 1), (1, 0, 1), (0, 0, 0), (1, 1, 0), (1, 1, 1)][k]
        structs.append((pos, np.zeros(n, np.int32), cell, pbc))
    batch = make_batch(structs)
    _, nl = _build(g, batch, 4.5, skin=0.5)
    ref = brute_force_neighbors(batch, np.float32(4.5) + np.float32(0.5))
    assert np.array_equal(gpu_list_triples(nl), oracle_triples(ref))
    _check_rev(nl)


def test_list_solid_with_skin():
    g = need_gpu()
    batch, params, spec = make_workload("solid", reps=(8, 8, 7))
    _, nl = _build(g, batch, 6.0, skin=1.0)
    ref = brute_force_neighbors(batch, 7.0)
    assert np.array_equal(gpu_list_triples(nl), oracle_triples(ref))
    _check_rev(nl)


def test_list_sampled_rows_full_liquid():
    g = need_gpu()
    batch, params, spec = make_workload("liquid")
    _, nl = _build(g, batch, 5.0)
    rows = np.arange(0, batch.n_atoms, 97)
    ref = brute_force_neighbors(batch, 5.0, rows=rows)
    t = gpu_list_triples(nl)
    got = t[np.isin(t[:, 0], rows)]
    assert np.array_equal(got, oracle_triples(ref))
    _check_rev(nl)


def test_capacity_overflow_reports_required_size():
    g = need_gpu()
    from paper_2505_22168_amd import _capi as A
    import ctypes as C
    batch, params, spec = make_workload("tiny")
    system = g.System.from_batch(batch, "cuda")
    small = g.NeighborList(batch.n_atoms, 100, system.device)
    small.cutoff = 5.0
    lib = A.load()
    sc = system.c()
    nb = lib.gmnn_neighbors_workspace_bytes(C.byref(sc), 5.0, 0.0)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    nc = small.c()
    st = lib.gmnn_build_neighbors(C.byref(sc), 5.0, 0.0, C.byref(nc), A.GMNN_SYNC, C.c_void_p(ws.data_ptr()), nb,
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == A.GMNN_ERR_CAPACITY
    assert small.n_pairs == brute_force_neighbors(batch, 5.0).n_pairs
    assert small.status & A.GMNN_FLAG_CAPACITY
    # too small a workspace is rejected before anything runs
    st = lib.gmnn_build_neighbors(C.byref(sc), 5.0, 0.0, C.byref(nc), A.GMNN_SYNC, C.c_void_p(ws.data_ptr()), 16,
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == A.GMNN_ERR_WORKSPACE


def test_coincident_atoms_flagged():
    g = need_gpu()
    from paper_2505_22168_amd import _capi as A
    pos = np.array([[1, 1, 1], [1, 1, 1], [2.5, 1, 1]], np.float32)
    batch = make_batch([(pos, np.zeros(3, np.int32), np.eye(3) * 12.0, (1, 1, 1))])
    system = g.System.from_batch(batch, "cuda")
    with pytest.raises(A.GMNNError) as e:
        g.build_neighbors(system, 3.0)
    assert e.value.status == A.GMNN_ERR_DEVICE_FLAG


def test_list_is_deterministic():
    g = need_gpu()
    batch, params, spec = make_workload("ensemble", n_structs=10)
    _, a = _build(g, batch, 5.0)
    _, b = _build(g, batch, 5.0)
    assert np.array_equal(gpu_list_triples(a), gpu_list_triples(b))
    assert torch.equal(a.rev[:a.n_pairs], b.rev[:b.n_pairs])
