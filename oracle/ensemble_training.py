"""Shallow-ensemble training step, plain FP64 definitions (test
infrastructure only: the product path never imports this module).

* Probabilistic losses of Section 2.2, eq. (nll): the Gaussian negative log
  likelihood and the closed-form continuous ranked probability score of a
  normal distribution, applied to the ensemble mean and the ensemble's
  population variance (1/M, as in the uncertainty equation).  The squared
  error of the mean is the homoscedastic reference.
* Loss terms of Section 3.4: an energy term and a force term, each weighted,
  the energy term optionally divided by the structure's atom count.
    L = w_E (1/B) sum_b l(x_b^1..M, x_b^ref) + w_F (1/(3N)) sum_{i,a} l(F_ia^1..M, F_ia^ref)
  with x_b^m = E_b^m (or E_b^m / N_b) and F^m = -dE^m/dx the per-head forces
  of eq. (jacobian).  Readings: forces are scored per Cartesian component,
  each with its own ensemble variance; var_floor is added to every
  variance (the paper leaves sigma -> 0 undefined); a structure without
  atoms adds nothing to a per-atom energy term.
* Adam (Kingma & Ba 2015, Algorithm 1) with the parameter groups of Section
  3.4 (embedding = beta, neural network = W1, b1, W2, b2, W3, b3, scale,
  shift: one learning rate each), and the learning-rate schedules Section
  3.4 names (linear decay, cyclic cosine).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .gmnn import DT, PARAM_NAMES, _tensors, pair_vectors, moments, invariants, mlp

GROUP_OF = {"beta": "embedding", "W1": "nn", "b1": "nn", "W2": "nn", "b2": "nn", "W3": "nn", "b3": "nn",
            "scale": "scale", "shift": "shift"}
GROUPS = ("embedding", "nn", "scale", "shift")


# ----------------------------------------------------------------------------
# losses (eq. nll)
# ----------------------------------------------------------------------------
def gaussian_nll(x_mean, x_ref, var):
    """Negative log likelihood of x_ref under N(x_mean, var), eq. (nll)."""
    return 0.5 * ((x_mean - x_ref) ** 2 / var + torch.log(2.0 * math.pi * var))


def gaussian_crps(x_mean, x_ref, var):
    """CRPS of N(x_mean, var) at x_ref, eq. (nll): sigma [z (2 Phi(z) - 1) +
    2 phi(z) - 1/sqrt(pi)] with z = |x_mean - x_ref| / sigma."""
    sigma = torch.sqrt(var)
    z = torch.abs(x_mean - x_ref) / sigma
    Phi = 0.5 * (1.0 + torch.erf(z / math.sqrt(2.0)))
    phi = torch.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return sigma * (z * (2.0 * Phi - 1.0) + 2.0 * phi - 1.0 / math.sqrt(math.pi))


def squared_error(x_mean, x_ref, var):
    """(x_mean - x_ref)^2; the variance plays no part."""
    return (x_mean - x_ref) ** 2


LOSSES = {"mse": squared_error, "nll": gaussian_nll, "crps": gaussian_crps}


@dataclass
class LossSpec:
    energy: str = "crps"
    force: str = "crps"
    w_energy: float = 1.0
    w_force: float = 1.0
    energy_per_atom: bool = True
    var_floor: float = 0.0


def ensemble_mean_var(x):
    """Mean and population variance over the last axis (the heads)."""
    mean = x.mean(-1)
    return mean, ((x - mean[..., None]) ** 2).mean(-1)


def ensemble_loss(E_heads, F_heads, E_ref, F_ref, n_atoms, spec: LossSpec):
    """The two terms (energy, force) of the loss; E_heads [B, M], F_heads
    [M, N, 3], E_ref [B], F_ref [N, 3], n_atoms [B] (torch float64)."""
    B = E_heads.shape[0]
    N = F_heads.shape[1]
    xE, xr = E_heads, E_ref
    keep = torch.ones(B, dtype=torch.bool)
    if spec.energy_per_atom:
        # a structure without atoms has no per-atom energy: it adds nothing
        # to the per-atom term (B still counts it)
        keep = n_atoms > 0
        na = torch.where(keep, n_atoms, torch.ones_like(n_atoms))
        xE, xr = E_heads / na[:, None], E_ref / na
    mE, vE = ensemble_mean_var(xE)
    lE = LOSSES[spec.energy](mE, xr, vE + spec.var_floor)
    LE = spec.w_energy / B * torch.where(keep, lE, torch.zeros_like(lE)).sum()
    mF, vF = ensemble_mean_var(F_heads.permute(1, 2, 0))             # [N, 3]
    LF = spec.w_force / (3 * N) * LOSSES[spec.force](mF, F_ref, vF + spec.var_floor).sum() if N else 0.0 * LE
    return LE, LF


def ensemble_loss_grads(E_heads, F_heads, E_ref, F_ref, n_atoms, spec: LossSpec):
    """(L_E, L_F, dL/dE^m [B, M], dL/dF^m [M, N, 3]) as numpy, by autograd."""
    E = torch.as_tensor(np.asarray(E_heads, dtype=np.float64)).requires_grad_(True)
    F = torch.as_tensor(np.asarray(F_heads, dtype=np.float64)).requires_grad_(True)
    LE, LF = ensemble_loss(E, F, torch.as_tensor(np.asarray(E_ref, dtype=np.float64)),
                           torch.as_tensor(np.asarray(F_ref, dtype=np.float64)),
                           torch.as_tensor(np.asarray(n_atoms, dtype=np.float64)), spec)
    gE, gF = torch.autograd.grad(LE + LF, (E, F), allow_unused=True)
    gE = np.zeros(E.shape) if gE is None else gE.numpy()
    gF = np.zeros(F.shape) if gF is None else gF.numpy()
    return float(LE.detach()), float(LF.detach()), gE, gF


@dataclass
class EnsembleStep:
    loss_energy: float
    loss_force: float
    energy_heads: np.ndarray     # [B, M]
    forces_heads: np.ndarray     # [M, N, 3]
    dL_dE: np.ndarray            # [B, M]
    dL_dF: np.ndarray            # [M, N, 3]
    grads: dict                  # parameter name -> dL/dtheta
    dL_dpos: np.ndarray          # [N, 3] gradient of the loss in the positions


def ensemble_loss_and_param_grads(batch, params, nl, E_ref, F_ref, spec: LossSpec) -> EnsembleStep:
    """Per-head energies and forces (eq. jacobian: one gradient per head),
    the loss of Section 3.4 with the terms of eq. (nll), and its gradient
    with respect to every parameter array."""
    p, pos0, cell, soa, sp, i, j, S = _tensors(batch, params, nl)
    p = {k: v.clone().requires_grad_(True) for k, v in p.items()}
    mspec = params.spec
    B, N, M = batch.n_structs, batch.n_atoms, mspec.n_heads
    pos = pos0.clone().requires_grad_(True)
    d = pair_vectors(pos, cell, soa, i, j, S)
    P = moments(d, i, sp[i], sp[j], p["beta"], mspec, N)
    G = invariants(*P)
    y = mlp(G, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"])
    Ei = p["scale"][sp][:, None] * y + p["shift"][sp][:, None]
    Eb = torch.zeros((B, M), dtype=DT).index_add(0, soa, Ei)
    Fh = torch.stack([-torch.autograd.grad(Eb[:, m].sum(), pos, create_graph=True)[0] for m in range(M)])
    nb = torch.as_tensor(np.diff(batch.atom_ptr), dtype=DT)
    LE, LF = ensemble_loss(Eb, Fh, torch.as_tensor(np.asarray(E_ref, dtype=np.float64)),
                           torch.as_tensor(np.asarray(F_ref, dtype=np.float64)), nb, spec)
    out = torch.autograd.grad(LE + LF, [p[k] for k in PARAM_NAMES] + [Eb, Fh, pos], allow_unused=True)
    grads = {k: (g.detach().numpy() if g is not None else np.zeros(p[k].shape)) for k, g in zip(PARAM_NAMES, out)}
    gE = out[len(PARAM_NAMES)]
    gF = out[len(PARAM_NAMES) + 1]
    return EnsembleStep(float(LE.detach()), float(LF.detach()), Eb.detach().numpy(), Fh.detach().numpy(),
                        np.zeros((B, M)) if gE is None else gE.detach().numpy(),
                        np.zeros((M, N, 3)) if gF is None else gF.detach().numpy(), grads,
                        out[len(PARAM_NAMES) + 2].detach().numpy())


# ----------------------------------------------------------------------------
# Adam with parameter groups, learning-rate schedules
# ----------------------------------------------------------------------------
def adam_step(params: dict, grads: dict, m1: dict, m2: dict, t: int, lr: dict, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (Kingma & Ba, Algorithm 1), in place on
    float64 numpy arrays: first and second moment estimates, their bias
    corrections, then theta -= lr_group * mhat / (sqrt(vhat) + eps).  lr maps a
    group name to its learning rate."""
    for k, g in grads.items():
        g = np.asarray(g, dtype=np.float64)
        m1[k] = beta1 * m1[k] + (1.0 - beta1) * g
        m2[k] = beta2 * m2[k] + (1.0 - beta2) * g * g
        mhat = m1[k] / (1.0 - beta1 ** t)
        vhat = m2[k] / (1.0 - beta2 ** t)
        params[k] = params[k] - lr[GROUP_OF[k]] * mhat / (np.sqrt(vhat) + eps)
    return params, m1, m2


def lr_factor(kind: str, step: int, total_steps: int = 1, end_factor: float = 0.0, period: int = 1,
              decay_factor: float = 1.0) -> float:
    """Multiplier of every group's base learning rate at a step (0-based).
    linear: from 1 down to end_factor over total_steps, then constant;
    cosine: cyclic cosine annealing, each cycle of `period` steps falling
    from its peak to 0 along half a cosine, the peak of cycle c being
    decay_factor^c; constant: 1."""
    if kind == "constant":
        return 1.0
    if kind == "linear":
        frac = min(step, total_steps) / total_steps
        return 1.0 + (end_factor - 1.0) * frac
    if kind == "cosine":
        c, r = divmod(step, period)
        return decay_factor ** c * 0.5 * (1.0 + math.cos(math.pi * r / period))
    raise ValueError(kind)
