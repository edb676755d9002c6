"""Batch active learning by last-layer gradient features (Section 2.4; test
infrastructure only).

  phi(S) = gradient of the head-mean energy of S w.r.t. the last layer
           (eq. lastlayer), here one head's weights and bias (the other
           heads' blocks repeat it), by autograd through the plain definition;
  greedy maximum-distance selection (eq. maxdist): repeatedly pick the pool
           entry whose smallest distance to the training entries and the
           entries picked so far is largest.  The paper's minimum runs over
           the pool and the batch, which would always be zero (the entry
           itself); read as the training set plus the batch.  With no
           training entries the first pick is the entry of largest norm.
           Ties go to the smaller index; distances in float64.
"""
from __future__ import annotations

import numpy as np
import torch

from .gmnn import DT, _tensors, atomic_energies


def last_layer_features(batch, params, nl):
    """[B, H2 + 1] float64: d(Ebar_b)/d(W3[:, 0]) and d(Ebar_b)/d(b3[0])."""
    p, *_ = _tensors(batch, params, nl)
    p = {k: v.clone().requires_grad_(k in ("W3", "b3")) for k, v in p.items()}
    E = atomic_energies(batch, params, nl, p=p)                     # [N, M]
    soa = torch.as_tensor(batch.struct_of_atom(), dtype=torch.long)
    Eb = torch.zeros((batch.n_structs, E.shape[1]), dtype=DT).index_add(0, soa, E).mean(1)
    rows = []
    for b in range(batch.n_structs):
        gW, gb = torch.autograd.grad(Eb[b], (p["W3"], p["b3"]), retain_graph=True)
        rows.append(torch.cat([gW[:, 0], gb[:1]]))
    return torch.stack(rows).numpy()


def max_distance_selection(pool, n_select, train=None):
    """Indices of the greedy maximum-distance picks, in order."""
    pool = np.asarray(pool, dtype=np.float64)
    chosen = []
    ref = [] if train is None else [np.asarray(t, dtype=np.float64) for t in np.asarray(train)]
    for _ in range(n_select):
        best, best_i = -1.0, -1
        for i in range(pool.shape[0]):
            if i in chosen:
                continue
            others = ref + [pool[c] for c in chosen]
            if others:
                score = min(float(((pool[i] - o) ** 2).sum()) for o in others)
            else:
                score = float((pool[i] ** 2).sum())
            if score > best:
                best, best_i = score, i
        chosen.append(best_i)
    return np.array(chosen, dtype=np.int64)
