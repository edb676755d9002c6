"""gmnn_energy_forces_noalloc (workspace in the library's fixed scratch
array) against gmnn_energy_forces (caller workspace) through the C ABI:
identical results on consecutive calls with shrinking inputs, and inputs
beyond the scratch limit rejected before anything runs."""
import ctypes as C

import numpy as np
import pytest
import torch

from workloads import make_workload
from gpu_helpers import gpu, need_gpu

pytestmark = gpu


def _setup(g, name, **kw):
    batch, params, spec = make_workload(name, **kw)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.model.r_cut, spec.skin)
    model = g.Model.from_params(params, "cuda")
    return system, nl, model


def _outputs(g, model, system):
    B, N, M = system.n_structs, system.n_atoms, model.spec.n_heads
    o = dict(energy=torch.full((B, M), float("nan"), dtype=torch.float64, device="cuda"),
             forces=torch.full((N, 3), float("nan"), dtype=torch.float32, device="cuda"),
             stress=torch.full((B, 3, 3), float("nan"), dtype=torch.float64, device="cuda"),
             atomic=torch.full((N, M), float("nan"), dtype=torch.float32, device="cuda"),
             mean=torch.full((B,), float("nan"), dtype=torch.float64, device="cuda"),
             status=torch.zeros(1, dtype=torch.int32, device="cuda"))
    from paper_2505_22168_amd import _capi as A
    p = lambda t: C.c_void_p(t.data_ptr())
    oc = A.gmnn_outputs(p(o["energy"]), p(o["forces"]), p(o["stress"]), None, None, p(o["atomic"]), p(o["mean"]),
                        p(o["status"]))
    return o, oc


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_matches_workspace_entry_point(precision):
    g = need_gpu()
    from paper_2505_22168_amd import _capi as A
    lib = A.load()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    flags = (A.GMNN_PREC_BF16 if precision == "bf16" else A.GMNN_PREC_FP32) | A.GMNN_WANT_STRESS
    # largest first (split schedule, chunked per-structure sums), then smaller
    # inputs (fused schedule) reusing the same scratch array
    for name, kw in [("solid", dict(reps=(22, 22, 18))), ("liquid", {}), ("tiny", {})]:
        system, nl, model = _setup(g, name, **kw)
        mc, sc, nc = model.c(), system.c(), nl.c()
        nbytes = lib.gmnn_workspace_bytes(A.GMNN_OP_ENERGY_FORCES, C.byref(mc), C.byref(sc), C.byref(nc), flags)
        assert 0 < nbytes <= A.GMNN_NOALLOC_SCRATCH_BYTES
        print(f"{name} {precision}: {system.n_atoms} atoms, workspace {nbytes / 2**20:.1f} MiB", flush=True)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        ref, rc = _outputs(g, model, system)
        A.check(lib.gmnn_energy_forces(C.byref(mc), C.byref(sc), C.byref(nc), flags, C.byref(rc),
                                       C.c_void_p(ws.data_ptr()), nbytes, stream), "gmnn_energy_forces")
        got, gc = _outputs(g, model, system)
        A.check(lib.gmnn_energy_forces_noalloc(C.byref(mc), C.byref(sc), C.byref(nc), flags | A.GMNN_SYNC,
                                               C.byref(gc), stream), "gmnn_energy_forces_noalloc")
        torch.cuda.synchronize()
        for k in ("energy", "forces", "stress", "atomic", "mean"):
            assert torch.isfinite(got[k]).all(), (name, k)
            assert torch.equal(got[k], ref[k]), (name, k)
        assert int(got["status"].item()) == 0


def test_noalloc_rejects_inputs_beyond_the_scratch_limit():
    g = need_gpu()
    from paper_2505_22168_amd import _capi as A
    lib = A.load()
    system, nl, model = _setup(g, "solid", reps=(40, 40, 30))  # 48,000 atoms
    mc, sc, nc = model.c(), system.c(), nl.c()
    nbytes = lib.gmnn_workspace_bytes(A.GMNN_OP_ENERGY_FORCES, C.byref(mc), C.byref(sc), C.byref(nc), 0)
    assert nbytes > A.GMNN_NOALLOC_SCRATCH_BYTES
    out, oc = _outputs(g, model, system)
    st = lib.gmnn_energy_forces_noalloc(C.byref(mc), C.byref(sc), C.byref(nc), 0, C.byref(oc),
                                        C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == A.GMNN_ERR_SCRATCH_LIMIT
    torch.cuda.synchronize()
    assert torch.isnan(out["energy"]).all()  # nothing ran
