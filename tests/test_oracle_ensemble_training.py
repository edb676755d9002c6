"""Pins of the oracle's shallow-ensemble training step (Section 2.2, eq. nll;
Section 3.4): the CRPS closed form against numerical integration of its
definition, the NLL against a library normal density, the losses' mean
derivatives in closed form, per-head parameter gradients against finite
differences and (one head, squared error) against the energy+force loss,
Adam with parameter groups against torch.optim.Adam, and the learning-rate
schedules at their defining points."""
import copy
import dataclasses
import math

import numpy as np
import pytest
import torch
from scipy import integrate, stats

from oracle import brute_force_neighbors, evaluate, loss_and_param_grads
from oracle.ensemble_training import (
    GROUP_OF, GROUPS, LossSpec, adam_step, ensemble_loss, ensemble_loss_and_param_grads, ensemble_loss_grads,
    ensemble_mean_var, gaussian_crps, gaussian_nll, lr_factor,
)
from oracle.gmnn import PARAM_NAMES
from workloads import make_workload
from workloads.configs import ModelSpec, make_params


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


@pytest.mark.parametrize("mu,sigma,y", [(0.0, 1.0, 0.3), (1.5, 0.2, 1.1), (-2.0, 3.0, 4.0), (0.7, 0.05, 0.7)])
def test_crps_closed_form_equals_its_integral_definition(mu, sigma, y):
    """CRPS(F, y) = int (F(t) - 1[t >= y])^2 dt for the normal CDF F."""
    F = lambda t: stats.norm.cdf(t, mu, sigma)
    lo, hi = min(mu, y) - 12 * sigma, max(mu, y) + 12 * sigma
    a, _ = integrate.quad(lambda t: F(t) ** 2, lo, y, epsabs=1e-13, epsrel=1e-12, limit=200)
    b, _ = integrate.quad(lambda t: (1 - F(t)) ** 2, y, hi, epsabs=1e-13, epsrel=1e-12, limit=200)
    got = float(gaussian_crps(_t(mu), _t(y), _t(sigma * sigma)))
    assert abs(got - (a + b)) < 1e-9 * max(1.0, a + b)


def test_crps_at_zero_error_and_nll_against_library_density():
    s = 0.37
    assert abs(float(gaussian_crps(_t(1.0), _t(1.0), _t(s * s))) - s * (math.sqrt(2) - 1) / math.sqrt(math.pi)) < 1e-15
    for mu, sigma, y in [(0.0, 1.0, 0.3), (2.0, 0.1, 1.7), (-1.0, 4.0, 3.0)]:
        want = -stats.norm.logpdf(y, mu, sigma)
        assert abs(float(gaussian_nll(_t(mu), _t(y), _t(sigma * sigma))) - want) < 1e-12 * max(1, abs(want))


def test_population_variance_matches_numpy():
    x = np.random.default_rng(0).normal(size=(5, 7))
    m, v = ensemble_mean_var(_t(x))
    assert np.allclose(m.numpy(), x.mean(1), rtol=0, atol=1e-15)
    assert np.allclose(v.numpy(), x.var(1, ddof=0), rtol=0, atol=1e-14)


@pytest.mark.parametrize("kind", ["nll", "crps", "mse"])
def test_head_gradients_sum_to_the_mean_derivative(kind):
    """The variance does not change when every head moves by the same amount,
    so sum_m dL/dx^m is the loss's derivative in the mean alone:
    CRPS 2 Phi(u/sigma) - 1, NLL u / sigma^2, squared error 2u."""
    rng = np.random.default_rng(3)
    B, M, N = 4, 6, 5
    E = rng.normal(size=(B, M)) * 0.3 - 10.0
    F = rng.normal(size=(M, N, 3))
    Er = rng.normal(size=B) * 0.3 - 10.0
    Fr = rng.normal(size=(N, 3))
    nb = np.array([3.0, 5.0, 4.0, 7.0])
    spec = LossSpec(kind, kind, w_energy=0.7, w_force=1.3, energy_per_atom=True)
    _, _, gE, gF = ensemble_loss_grads(E, F, Er, Fr, nb, spec)
    xm, xr = E.mean(1) / nb, Er / nb
    v = E.var(1) / nb ** 2
    u = xm - xr
    d = {"crps": 2 * stats.norm.cdf(u / np.sqrt(v)) - 1, "nll": u / v, "mse": 2 * u}[kind]
    assert np.allclose(gE.sum(1), 0.7 / B * d / nb, rtol=1e-10, atol=1e-14)
    uF = F.mean(0) - Fr
    vF = F.var(0)
    dF = {"crps": 2 * stats.norm.cdf(uF / np.sqrt(vF)) - 1, "nll": uF / vF, "mse": 2 * uF}[kind]
    assert np.allclose(gF.sum(0), 1.3 / (3 * N) * dF, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("kind", ["nll", "crps"])
def test_head_gradients_match_central_differences(kind):
    rng = np.random.default_rng(4)
    E = rng.normal(size=(3, 4))
    F = rng.normal(size=(4, 2, 3))
    Er, Fr, nb = rng.normal(size=3), rng.normal(size=(2, 3)), np.array([2.0, 3.0, 1.0])
    spec = LossSpec(kind, kind, energy_per_atom=False, var_floor=1e-3)
    _, _, gE, gF = ensemble_loss_grads(E, F, Er, Fr, nb, spec)

    def L(E_, F_):
        a, b = ensemble_loss(_t(E_), _t(F_), _t(Er), _t(Fr), _t(nb), spec)
        return float(a + b)

    h = 1e-6
    for (b, m) in [(0, 0), (1, 3), (2, 1)]:
        Ep, Em = E.copy(), E.copy()
        Ep[b, m] += h
        Em[b, m] -= h
        assert abs((L(Ep, F) - L(Em, F)) / (2 * h) - gE[b, m]) < 1e-7
    for (m, i, a) in [(0, 0, 0), (3, 1, 2), (2, 0, 1)]:
        Fp, Fm = F.copy(), F.copy()
        Fp[m, i, a] += h
        Fm[m, i, a] -= h
        assert abs((L(E, Fp) - L(E, Fm)) / (2 * h) - gF[m, i, a]) < 1e-7


@pytest.fixture(scope="module")
def heads_setup():
    b, _, s = make_workload("train", n_structs=2, n_lo=12, n_hi=18)
    spec = ModelSpec(n_species=5, r_cut=5.0, hidden=(16, 16), n_heads=4, psi_scale=s.model.psi_scale)
    p = make_params(spec, 11)
    t = make_params(dataclasses.replace(spec, n_heads=1), 111)
    nl = brute_force_neighbors(b, 5.0)
    rt = evaluate(b, t, nl)
    return b, p, nl, rt.energy_mean, rt.forces


def test_per_head_forces_are_head_energy_gradients(heads_setup):
    """F^m of the training step equals the oracle's force of a one-head model
    made of head m alone."""
    b, p, nl, Er, Fr = heads_setup
    st = ensemble_loss_and_param_grads(b, p, nl, Er, Fr, LossSpec())
    for m in (0, 3):
        q = copy.deepcopy(p)
        q.spec = dataclasses.replace(p.spec, n_heads=1)
        q.W3 = p.W3[:, m:m + 1].copy()
        q.b3 = p.b3[m:m + 1].copy()
        r = evaluate(b, q, nl)
        assert np.abs(st.forces_heads[m] - r.forces).max() < 1e-10
        assert np.abs(st.energy_heads[:, m] - r.energy[:, 0]).max() < 1e-10


@pytest.mark.parametrize("kind", ["crps", "nll"])
def test_parameter_gradients_directional_differences(heads_setup, kind):
    b, p, nl, Er, Fr = heads_setup
    spec = LossSpec(kind, kind, w_energy=1.0, w_force=0.5, energy_per_atom=True, var_floor=1e-4)
    st = ensemble_loss_and_param_grads(b, p, nl, Er, Fr, spec)
    rng = np.random.default_rng(9)
    v = {k: rng.normal(size=np.shape(getattr(p, k))) for k in PARAM_NAMES}
    dirderiv = sum(float((st.grads[k] * v[k]).sum()) for k in PARAM_NAMES)

    def L(sign, h):
        q = copy.deepcopy(p)
        for k in PARAM_NAMES:
            setattr(q, k, getattr(p, k) + sign * h * v[k])
        s2 = ensemble_loss_and_param_grads(b, q, nl, Er, Fr, spec)
        return s2.loss_energy + s2.loss_force

    # five-point central difference (the NLL's curvature makes the
    # three-point one's h^2 error visible at 1e-6 relative)
    h = 1e-5
    fd = (8 * (L(1, h) - L(-1, h)) - (L(1, 2 * h) - L(-1, 2 * h))) / (12 * h)
    assert abs(fd - dirderiv) < 1e-7 * max(1.0, abs(dirderiv))


def test_one_head_squared_error_equals_energy_force_loss():
    """With one head and the squared error per atom, the ensemble step is the
    energy+force loss of the head-mean training path."""
    b, _, s = make_workload("train", n_structs=2, n_lo=12, n_hi=18)
    spec = ModelSpec(n_species=5, r_cut=5.0, hidden=(16, 16), n_heads=1, psi_scale=s.model.psi_scale)
    p = make_params(spec, 12)
    nl = brute_force_neighbors(b, 5.0)
    rt = evaluate(b, make_params(spec, 112), nl)
    L, g, dE, dF = loss_and_param_grads(b, p, nl, rt.energy_mean, rt.forces)
    st = ensemble_loss_and_param_grads(b, p, nl, rt.energy_mean, rt.forces, LossSpec("mse", "mse"))
    assert abs(st.loss_energy + st.loss_force - L) < 1e-12 * max(1, L)
    for k in PARAM_NAMES:
        assert np.allclose(st.grads[k], g[k], rtol=1e-9, atol=1e-13), k
    assert np.allclose(st.dL_dE[:, 0], dE, rtol=1e-10, atol=1e-15)
    assert np.allclose(st.dL_dF[0], dF, rtol=1e-10, atol=1e-15)


def test_adam_with_groups_matches_torch():
    """Four parameter groups with their own learning rates (one frozen at 0)
    over five steps agree with torch.optim.Adam on float64 tensors."""
    rng = np.random.default_rng(5)
    shapes = {"beta": (2, 2, 5, 7), "W1": (6, 4), "b1": (4,), "W2": (4, 4), "b2": (4,), "W3": (4, 3), "b3": (3,),
              "scale": (2,), "shift": (2,)}
    lr = {"embedding": 0.0, "nn": 1e-2, "scale": 3e-3, "shift": 5e-2}
    params = {k: rng.normal(size=s) for k, s in shapes.items()}
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in params.items()}
    groups = [{"params": [tp[k] for k in PARAM_NAMES if GROUP_OF[k] == g], "lr": lr[g]} for g in GROUPS]
    opt = torch.optim.Adam(groups, betas=(0.9, 0.999), eps=1e-8)
    m1 = {k: np.zeros(s) for k, s in shapes.items()}
    m2 = {k: np.zeros(s) for k, s in shapes.items()}
    start = copy.deepcopy(params)
    for t in range(1, 6):
        g = {k: rng.normal(size=s) * 10.0 ** rng.integers(-3, 2) for k, s in shapes.items()}
        for k in shapes:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
        params, m1, m2 = adam_step(params, g, m1, m2, t, lr)
    for k in shapes:
        assert np.allclose(params[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14), k
    assert np.array_equal(params["beta"], start["beta"])


def test_first_adam_step_moves_each_entry_by_its_learning_rate():
    """At t = 1 the bias-corrected update is lr * g / (|g| + eps): every entry
    with |g| >> eps moves by lr against the sign of its gradient."""
    p = {"W1": np.zeros(5)}
    g = {"W1": np.array([3.0, -0.2, 1e-3, -7.0, 0.5])}
    p, _, _ = adam_step(p, g, {"W1": np.zeros(5)}, {"W1": np.zeros(5)}, 1, {"nn": 0.1}, eps=1e-12)
    assert np.allclose(p["W1"], -0.1 * np.sign(g["W1"]), rtol=1e-8, atol=0)


def test_learning_rate_schedules_at_their_defining_points():
    assert lr_factor("constant", 123) == 1.0
    assert lr_factor("linear", 0, total_steps=100, end_factor=0.1) == 1.0
    assert abs(lr_factor("linear", 100, total_steps=100, end_factor=0.1) - 0.1) < 1e-15
    assert abs(lr_factor("linear", 250, total_steps=100, end_factor=0.1) - 0.1) < 1e-15
    assert abs(lr_factor("linear", 50, total_steps=100, end_factor=0.0) - 0.5) < 1e-15
    # cyclic cosine: a full peak at each cycle start, half of it mid-cycle,
    # the peak shrinking by decay_factor per cycle
    assert lr_factor("cosine", 0, period=40, decay_factor=0.95) == 1.0
    assert abs(lr_factor("cosine", 20, period=40, decay_factor=0.95) - 0.5) < 1e-15
    assert abs(lr_factor("cosine", 80, period=40, decay_factor=0.95) - 0.95 ** 2) < 1e-15
    assert abs(lr_factor("cosine", 100, period=40, decay_factor=0.95) - 0.5 * 0.95 ** 2) < 1e-15
    assert lr_factor("cosine", 39, period=40) < 1e-2


def test_position_gradient_of_the_ensemble_loss(heads_setup):
    """dL/dx of the ensemble loss (per-head forces inside) against five-point
    differences along a random displacement; zero net gradient."""
    b, p, _, Er, Fr = heads_setup
    nl = brute_force_neighbors(b, 5.5)
    spec = LossSpec("crps", "nll", var_floor=1e-4)
    st = ensemble_loss_and_param_grads(b, p, nl, Er, Fr, spec)
    assert np.abs(st.dL_dpos.sum(0)).max() < 1e-10 * max(1.0, np.abs(st.dL_dpos).max())
    v = np.random.default_rng(6).normal(size=b.pos.shape)
    ana = float((st.dL_dpos * v).sum())

    def L(t):
        bt = dataclasses.replace(b, pos=b.pos.astype(np.float64) + t * v)
        s2 = ensemble_loss_and_param_grads(bt, p, nl, Er, Fr, spec)
        return s2.loss_energy + s2.loss_force

    h = 1e-4
    fd = (8 * (L(h) - L(-h)) - (L(2 * h) - L(-2 * h))) / (12 * h)
    assert abs(fd - ana) < 1e-6 * max(1.0, abs(ana)), (fd, ana)


def test_empty_structure_adds_nothing_to_the_per_atom_energy_term():
    """Dropping a structure without atoms from the batch changes the per-atom
    energy term only through the 1/B prefactor."""
    rng = np.random.default_rng(12)
    E = rng.normal(size=(4, 3)) - 5.0
    E[2] = 0.0
    Er = rng.normal(size=4) - 5.0
    F = rng.normal(size=(3, 6, 3))
    Fr = rng.normal(size=(6, 3))
    nb = np.array([2.0, 3.0, 0.0, 1.0])
    spec = LossSpec("crps", "nll", var_floor=1e-3)
    LE, LF, gE, _ = ensemble_loss_grads(E, F, Er, Fr, nb, spec)
    keep = [0, 1, 3]
    LE3, LF3, gE3, _ = ensemble_loss_grads(E[keep], F, Er[keep], Fr, nb[keep], spec)
    assert np.isfinite(LE) and abs(LE * 4 - LE3 * 3) < 1e-12
    assert abs(LF - LF3) < 1e-15
    assert np.all(gE[2] == 0.0) and np.allclose(gE[keep] * 4, gE3 * 3, rtol=1e-12, atol=0)
