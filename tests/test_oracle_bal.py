"""Pins of the oracle's batch-active-learning pieces (Section 2.4):
last-layer gradient features against a hand-derived closed form and finite
differences, and the greedy maximum-distance selection against an exhaustive
check of every pick on small pools."""
import copy
import itertools

import numpy as np
import torch

from oracle import brute_force_neighbors, evaluate, last_layer_features, max_distance_selection
from workloads import make_workload


def _swish(x):
    return x / (1.0 + np.exp(-x))


def test_features_closed_form_with_constant_second_layer():
    """W2 = 0: every atom's h2 = swish(b2), so the gradient of the head-mean
    energy w.r.t. W3[:, 0] is (1/M) swish(b2) sum_i sigma_Zi and w.r.t.
    b3[0] is (1/M) sum_i sigma_Zi."""
    batch, params, spec = make_workload("ensemble", n_structs=3)
    p = copy.deepcopy(params)
    p.W2 = np.zeros_like(p.W2)
    nl = brute_force_neighbors(batch, 5.0)
    phi = last_layer_features(batch, p, nl)
    M = p.spec.n_heads
    for b in range(batch.n_structs):
        ssum = p.scale[batch.species[batch.atom_ptr[b]:batch.atom_ptr[b + 1]]].sum()
        want = np.concatenate([_swish(p.b2) * ssum, [ssum]]) / M
        assert np.allclose(phi[b], want, rtol=1e-12, atol=1e-12)


def test_features_are_finite_differences_of_the_energy():
    batch, params, spec = make_workload("ensemble", n_structs=2)
    nl = brute_force_neighbors(batch, 5.0)
    phi = last_layer_features(batch, params, nl)
    h = 1e-6
    for k in (0, 7, params.W3.shape[0] - 1):
        e = []
        for sgn in (1, -1):
            q = copy.deepcopy(params)
            q.W3[k, 0] += sgn * h
            e.append(evaluate(batch, q, nl, want_stress=False).energy_mean)
        fd = (e[0] - e[1]) / (2 * h)
        assert np.allclose(fd, phi[:, k], rtol=1e-6, atol=1e-8)


def _check_greedy(pool, chosen, train):
    """Every pick maximises the smallest distance to the training entries and
    the earlier picks, over the entries not yet picked (exhaustive)."""
    ref = [] if train is None else list(train)
    for s, c in enumerate(chosen):
        others = ref + [pool[x] for x in chosen[:s]]
        def score(i):
            if not others:
                return float((pool[i] ** 2).sum())
            return min(float(((pool[i] - o) ** 2).sum()) for o in others)
        rest = [i for i in range(len(pool)) if i not in chosen[:s]]
        best = max(score(i) for i in rest)
        assert score(c) == best
        assert c == min(i for i in rest if score(i) == best)  # ties: smallest index


def test_selection_greedy_exhaustive_small_pools():
    rng = np.random.default_rng(0)
    for n, d, t in [(12, 3, 0), (15, 4, 3), (9, 2, 1)]:
        pool = rng.normal(size=(n, d))
        train = rng.normal(size=(t, d)) if t else None
        chosen = max_distance_selection(pool, 6, train)
        assert len(set(chosen.tolist())) == 6
        _check_greedy(pool, chosen.tolist(), train)


def test_selection_line_points_by_hand():
    """Points 0, 1, 2, 10 on a line, no training set: the largest norm (10)
    first, then the point farthest from it (0), then 2 (distance 2 to 0 and
    8 to 10 beats 1's distance 1)."""
    pool = np.array([[1.0], [0.0], [10.0], [2.0]])
    assert max_distance_selection(pool, 3).tolist() == [2, 1, 3]
    # with a training entry at 9 the farthest from it goes first
    assert max_distance_selection(pool, 1, train=np.array([[9.0]])).tolist() == [1]
