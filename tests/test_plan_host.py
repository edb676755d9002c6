"""Execution-plan resolution (host-only C code) and the autotune cache file.

gmnn_resolve_plan reads only host-side fields (shapes, the host copies of
atom_ptr / cell), so it runs here without a device: the device pointers are
placeholders that the call never dereferences."""
import ctypes as C
import json

import numpy as np
import pytest

from paper_2505_22168_amd import _capi as A

FAKE = C.c_void_p(0x1000)  # stands in for device pointers; never read


def _model(n_species=5, hidden=256, heads=1):
    return A.gmnn_model(n_species, 5, 7, hidden, hidden, heads, 0.5, 5.0, 1.0, 0.1,
                        FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE)


class _Sys:
    def __init__(self, sizes):
        self.ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        B = len(sizes)
        self.cell = np.tile(np.eye(3) * 20.0, (B, 1, 1)).astype(np.float64)
        self.pbc = np.ones((B, 3), np.uint8)
        self.c = A.gmnn_system(B, int(self.ptr[-1]), FAKE, self.ptr.ctypes.data_as(C.c_void_p), FAKE, FAKE,
                               FAKE, self.cell.ctypes.data_as(C.c_void_p), FAKE, self.pbc.ctypes.data_as(C.c_void_p))


def _resolve(model, sysobj, flags, sched=None, lanes=0, readout=0, full=False, ta=0):
    lib = A.load()
    out = A.gmnn_plan()
    plan = None if sched is None else C.byref(A.gmnn_plan(sched, lanes, readout, ta))
    st = lib.gmnn_resolve_plan(C.byref(model), C.byref(sysobj.c), flags, plan, C.byref(out))
    if full:
        return st, (out.schedule, out.lanes_per_atom, out.readout, out.tile_atoms)
    return st, (out.schedule, out.lanes_per_atom)


def test_builtin_plan_small_and_large():
    m = _model()
    assert _resolve(m, _Sys([1536]), 0) == (A.GMNN_OK, (A.GMNN_SCHEDULE_FUSED, 64))
    assert _resolve(m, _Sys([100000]), 0) == (A.GMNN_OK, (A.GMNN_SCHEDULE_SPLIT, 16))
    # force variance needs one backward per head: the fused tile does not serve it
    assert _resolve(m, _Sys([1536]), A.GMNN_WANT_FORCE_VAR) == (A.GMNN_OK, (A.GMNN_SCHEDULE_SPLIT, 64))
    assert A.load().gmnn_uses_fused_path(C.byref(m), C.byref(_Sys([1536]).c), 0) == 1


def test_explicit_plans():
    m = _model()
    small = _Sys([120] * 30)
    for lanes in (8, 16, 32, 64):
        assert _resolve(m, small, 0, A.GMNN_SCHEDULE_SPLIT, lanes) == (A.GMNN_OK, (A.GMNN_SCHEDULE_SPLIT, lanes))
        assert _resolve(m, small, A.GMNN_PREC_BF16, A.GMNN_SCHEDULE_FUSED, lanes)[0] == A.GMNN_OK
    # the fused tile on a large batch of small structures is allowed (one
    # reduction chunk per structure) ...
    assert _resolve(m, _Sys([200] * 100), 0, A.GMNN_SCHEDULE_FUSED, 16)[0] == A.GMNN_OK
    # ... but not for a structure above the fused schedule's limit
    assert _resolve(m, _Sys([16385]), 0, A.GMNN_SCHEDULE_FUSED, 16)[0] == A.GMNN_ERR_UNSUPPORTED
    assert _resolve(m, _Sys([16384]), 0, A.GMNN_SCHEDULE_FUSED, 16)[0] == A.GMNN_OK
    assert _resolve(m, small, A.GMNN_WANT_FORCE_VAR, A.GMNN_SCHEDULE_FUSED, 0)[0] == A.GMNN_ERR_UNSUPPORTED
    assert _resolve(_model(n_species=9), small, 0, A.GMNN_SCHEDULE_FUSED, 0)[0] == A.GMNN_ERR_UNSUPPORTED
    assert _resolve(_model(n_species=9), small, 0)[1][0] == A.GMNN_SCHEDULE_SPLIT


def test_readout_choice():
    m = _model(hidden=512)
    TILE, STREAM = A.GMNN_READOUT_TILE, A.GMNN_READOUT_STREAM
    SPLIT, FUSED = A.GMNN_SCHEDULE_SPLIT, A.GMNN_SCHEDULE_FUSED
    # built-in: fused below 16384 atoms (BF16 2x512 fits the fused tile's LDS,
    # FP32 2x512 does not), split with the streamed readout from there on
    assert _resolve(m, _Sys([12000]), A.GMNN_PREC_BF16, full=True) == (A.GMNN_OK, (FUSED, 64, TILE, 16))
    assert _resolve(m, _Sys([12000]), 0, full=True) == (A.GMNN_OK, (SPLIT, 16, TILE, 0))
    assert _resolve(m, _Sys([12000]), 0, SPLIT, full=True) == (A.GMNN_OK, (SPLIT, 16, TILE, 0))
    assert _resolve(m, _Sys([6000]), 0, SPLIT, full=True) == (A.GMNN_OK, (SPLIT, 64, TILE, 0))
    assert _resolve(m, _Sys([100000]), A.GMNN_PREC_BF16, full=True) == (A.GMNN_OK, (SPLIT, 16, STREAM, 0))
    assert _resolve(_model(), _Sys([1536]), 0, full=True)[1] == (FUSED, 64, TILE, 8)
    # force variance needs one backward per head: the tile readout only
    assert _resolve(_model(), _Sys([100000]), A.GMNN_WANT_FORCE_VAR, full=True)[1] == (SPLIT, 16, TILE, 0)
    assert _resolve(m, _Sys([200]), A.GMNN_WANT_FORCE_VAR, SPLIT, 16, STREAM)[0] == A.GMNN_ERR_UNSUPPORTED
    # the streamed readout belongs to the split schedule
    assert _resolve(m, _Sys([200]), 0, FUSED, 16, STREAM)[0] == A.GMNN_ERR_UNSUPPORTED
    assert _resolve(m, _Sys([200]), 0, SPLIT, 32, STREAM, full=True) == (A.GMNN_OK, (SPLIT, 32, STREAM, 0))
    assert _resolve(m, _Sys([100000]), 0, SPLIT, 16, TILE, full=True) == (A.GMNN_OK, (SPLIT, 16, TILE, 0))
    # sixteen heads fit the network block's LDS at every width and precision
    for hidden in (64, 256, 512):
        for flags in (0, A.GMNN_PREC_BF16):
            assert _resolve(_model(hidden=hidden, heads=16), _Sys([200]), flags, SPLIT, 16, STREAM)[0] == A.GMNN_OK
    assert _resolve(m, _Sys([200]), 0, SPLIT, 16, 5)[0] == A.GMNN_ERR_INVALID_ARG


def test_fused_tile_atoms():
    m = _model()
    FUSED, SPLIT, TILE = A.GMNN_SCHEDULE_FUSED, A.GMNN_SCHEDULE_SPLIT, A.GMNN_READOUT_TILE
    # built-in: 8-atom tiles while 16-atom ones would number fewer than the 256 compute units
    assert _resolve(m, _Sys([4080]), 0, full=True)[1] == (FUSED, 64, TILE, 8)
    assert _resolve(m, _Sys([4096]), 0, full=True)[1] == (FUSED, 64, TILE, 16)
    for ta in (8, 16):
        assert _resolve(m, _Sys([1536]), 0, FUSED, 32, 0, full=True, ta=ta) == (A.GMNN_OK, (FUSED, 32, TILE, ta))
        # tile sizes belong to the fused schedule
        assert _resolve(m, _Sys([1536]), 0, SPLIT, 16, 0, ta=ta)[0] == A.GMNN_ERR_UNSUPPORTED
        assert _resolve(m, _Sys([100000]), 0, 0, 0, 0, ta=ta)[0] == A.GMNN_ERR_UNSUPPORTED
    assert _resolve(m, _Sys([1536]), 0, FUSED, 32, 0, ta=12)[0] == A.GMNN_ERR_INVALID_ARG
    assert A.gmnn_plan.of({"schedule": 1, "lanes_per_atom": 32}).as_dict() == {
        "schedule": 1, "lanes_per_atom": 32, "readout": 0, "tile_atoms": 0}
    assert A.gmnn_plan.of((2, 16, 2)).as_dict()["readout"] == 2


def test_invalid_plans():
    m = _model()
    s = _Sys([100])
    assert _resolve(m, s, 0, A.GMNN_SCHEDULE_SPLIT, 12)[0] == A.GMNN_ERR_INVALID_ARG
    assert _resolve(m, s, 0, 7, 16)[0] == A.GMNN_ERR_INVALID_ARG
    lib = A.load()
    assert lib.gmnn_resolve_plan(None, C.byref(s.c), 0, None, None) == A.GMNN_ERR_INVALID_ARG
    best = A.gmnn_plan()
    assert lib.gmnn_autotune(C.byref(m), C.byref(s.c), None, 0, None, None, 0, None, 0, C.byref(best), None, 0,
                             None) == A.GMNN_ERR_INVALID_ARG


def test_tune_cache_roundtrip(tmp_path):
    from paper_2505_22168_amd.autotune import TuneCache, _pow2
    path = str(tmp_path / "sub" / "tune.json")
    c = TuneCache(path)
    assert c.get("k") is None
    c.put("k", {"schedule": 2, "lanes_per_atom": 32, "table": [[2, 32, 10.0, 9.0]]})
    c2 = TuneCache(path)
    assert c2.get("k")["lanes_per_atom"] == 32
    assert json.load(open(path))["k"]["schedule"] == 2
    assert [_pow2(x) for x in (0, 1, 3, 5, 1536, 100000)] == [0, 1, 4, 4, 2048, 131072]
