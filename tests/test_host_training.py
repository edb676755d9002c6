"""Host logic of the training step that runs without a GPU: the learning-rate
schedules of the C library (gmnn_lr_factor) against the oracle's, and its
refusal of invalid schedules."""
import math

import pytest

from oracle.ensemble_training import lr_factor as oracle_lr_factor


@pytest.fixture(scope="module")
def g():
    import paper_2505_22168_amd as g
    g.load_library()
    return g


@pytest.mark.parametrize("kw", [dict(kind="constant"), dict(kind="linear", total_steps=37, end_factor=0.05),
                                dict(kind="linear", total_steps=1, end_factor=2.0),
                                dict(kind="cosine", period=13, decay_factor=0.95),
                                dict(kind="cosine", period=1, decay_factor=0.5)])
def test_library_schedules_match_oracle(g, kw):
    for step in list(range(0, 60)) + [1000, 12345]:
        assert abs(g.lr_factor(step=step, **kw) - oracle_lr_factor(step=step, **kw)) < 1e-14


def test_invalid_schedules_give_nan(g):
    assert math.isnan(g.lr_factor("linear", 3, total_steps=0))
    assert math.isnan(g.lr_factor("cosine", 3, period=0))
    assert math.isnan(g.lr_factor("constant", -1))


def test_one_head_probabilistic_loss_without_floor_is_rejected(g):
    """With one head the ensemble variance is zero: a weighted NLL or CRPS term
    needs var_floor > 0, and gmnn_ensemble_loss refuses it before touching any
    buffer (host-side validation; no GPU call is made)."""
    import ctypes as C
    from paper_2505_22168_amd import _capi as A
    lib = A.load()
    dummy = (C.c_double * 4)()
    ptr = C.cast(dummy, C.c_void_p)
    sys_ = A.gmnn_system(n_structs=1, n_atoms=0, atom_ptr=ptr, atom_ptr_host=ptr)
    for kind in (A.GMNN_LOSS_NLL, A.GMNN_LOSS_CRPS):
        spec = A.gmnn_loss(energy_kind=kind, force_kind=A.GMNN_LOSS_MSE, w_energy=1.0, w_force=0.0, var_floor=0.0)
        st = lib.gmnn_ensemble_loss(C.byref(spec), C.byref(sys_), 1, ptr, None, ptr, None, ptr, None, None, None, 0,
                                    None)
        assert st == A.GMNN_ERR_INVALID_ARG
