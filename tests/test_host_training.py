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
