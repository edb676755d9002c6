"""Batch active learning (Section 2.4) on the GPU: last-layer gradient
features against the FP64 oracle (split schedule, both readouts), and the
greedy maximum-distance selection bit-exact against the oracle's on seeded
feature pools (FP64 distances on both sides)."""
import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors, last_layer_features, max_distance_selection
from workloads import make_workload
from gpu_helpers import gpu, need_gpu

pytestmark = gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("name,kw", [("ensemble", dict(n_structs=12)), ("train", dict(n_structs=3, n_lo=100, n_hi=200))])
def test_last_layer_features_match_oracle(name, kw, precision):
    g = need_gpu()
    batch, params, spec = make_workload(name, **kw)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.model.r_cut)
    model = g.Model.from_params(params, "cuda")
    phi = g.last_layer_features(model, system, nl, precision=precision).cpu().numpy()
    ref = last_layer_features(batch, params, brute_force_neighbors(batch, spec.model.r_cut))
    assert phi.shape == ref.shape
    rel = np.abs(phi - ref).max() / np.abs(ref).max()
    print(f"{name} {precision}: features max rel err {rel:.2e}")
    assert rel < (1e-5 if precision == "fp32" else 1e-4)


@pytest.mark.parametrize("n,d,t,b", [(300, 7, 0, 40), (2000, 257, 5, 25), (777, 33, 1, 777)])
def test_selection_matches_oracle(n, d, t, b):
    g = need_gpu()
    rng = np.random.default_rng(n + d)
    pool = rng.normal(size=(n, d)) * rng.uniform(0.5, 2.0, size=(n, 1))
    train = rng.normal(size=(t, d)) if t else None
    got = g.select_max_distance(torch.as_tensor(pool, device="cuda"), b,
                                None if train is None else torch.as_tensor(train, device="cuda")).cpu().numpy()
    if b <= 60:
        ref = max_distance_selection(pool, b, train)
        assert np.array_equal(got, ref), (got[:10], ref[:10])
    else:
        # the whole pool: a permutation whose first picks agree with the oracle
        assert sorted(got.tolist()) == list(range(n))
        assert np.array_equal(got[:20], max_distance_selection(pool, 20, train))


def test_selection_on_model_features():
    """End to end: features of 40 structures on the GPU, then 8 picks.  On
    the oracle's own features every pick is greedy-optimal up to the
    features' FP32 error (its smallest distance to the earlier picks is the
    largest one within 1e-4 relative)."""
    g = need_gpu()
    batch, params, spec = make_workload("ensemble", n_structs=40)
    system = g.System.from_batch(batch, "cuda")
    nl = g.build_neighbors(system, spec.model.r_cut)
    model = g.Model.from_params(params, "cuda")
    phi = g.last_layer_features(model, system, nl)
    got = g.select_max_distance(phi, 8).cpu().numpy().tolist()
    ref = last_layer_features(batch, params, brute_force_neighbors(batch, spec.model.r_cut))
    assert len(set(got)) == 8
    for s, c in enumerate(got):
        def score(i):
            if s == 0:
                return float((ref[i] ** 2).sum())
            return min(float(((ref[i] - ref[x]) ** 2).sum()) for x in got[:s])
        best = max(score(i) for i in range(len(ref)) if i not in got[:s])
        assert score(c) >= best * (1 - 1e-4)
