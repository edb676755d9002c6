"""Pins of the oracle's Bessel-like radial basis (Section 2.1 names the
non-orthogonal Bessel-like functions of Kocer et al. beside the Gaussians;
the formula is a reading, see oracle.gmnn.bessel_basis): hand-evaluated
values, vanishing value and slope at the cutoff, the r -> 0 limit, and the
energy/force consistency of a model built on it."""
import dataclasses
import math

import numpy as np
import torch

from oracle import brute_force_neighbors, evaluate
from oracle.gmnn import bessel_basis
from workloads import make_workload
from workloads.configs import make_params

RC = 5.0


def test_hand_values_at_half_cutoff():
    # x = pi/2: sinc(pi/2) = 2/pi, sinc(pi) = 0, sinc(3 pi/2) = -2/(3 pi)
    f = bessel_basis(torch.tensor([RC / 2], dtype=torch.float64), RC, 3)[0].numpy()
    f0 = 4.0 * math.sqrt(2.0) / (math.sqrt(5.0) * RC ** 1.5)        # a_0 * 2/pi
    f1 = 4.0 * math.sqrt(2.0) / (math.sqrt(13.0) * RC ** 1.5)       # a_1 * (-2/(3 pi)), a_1 < 0
    # n = 2: sinc(3 pi/2) + sinc(2 pi) = -2/(3 pi); a_2 = sqrt2 pi rc^-1.5 * 12/5
    f2 = -math.sqrt(2.0) * 12.0 / 5.0 * 2.0 / 3.0 / RC ** 1.5
    assert np.allclose(f, [f0, f1, f2], rtol=1e-13, atol=0)


def test_vanishes_with_zero_slope_at_cutoff():
    K = 7
    r = torch.tensor([RC], dtype=torch.complex128) + 1j * 1e-30
    f = bessel_basis(r, RC, K)
    assert np.abs(f.real.numpy()).max() < 1e-14
    slope = f.imag.numpy() / 1e-30          # complex-step derivative
    assert np.abs(slope).max() < 1e-14
    # but not inside: slopes of order one at r_c / 3
    r2 = torch.tensor([RC / 3], dtype=torch.complex128) + 1j * 1e-30
    assert np.abs(bessel_basis(r2, RC, K).imag.numpy() / 1e-30).min() > 1e-3


def test_small_r_limit():
    K = 7
    f = bessel_basis(torch.tensor([1e-7], dtype=torch.float64), RC, K)[0].numpy()
    n = np.arange(K)
    a = (-1.0) ** n * math.sqrt(2.0) * math.pi * RC ** -1.5 * (n + 1) * (n + 2) / np.sqrt((n + 1) ** 2 + (n + 2) ** 2)
    assert np.allclose(f, 2.0 * a, rtol=1e-10)


def _bessel_model(name, **kw):
    batch, params, spec = make_workload(name, **kw)
    s2 = dataclasses.replace(spec.model, basis="bessel", hidden=(32, 32))
    return batch, make_params(s2, 21), s2


def test_bessel_model_forces_are_energy_gradients():
    batch, params, spec = _bessel_model("tiny")
    nl = brute_force_neighbors(batch, spec.r_cut)
    r = evaluate(batch, params, nl)
    rng = np.random.default_rng(3)
    h = 1e-5
    for _ in range(4):
        k, a = int(rng.integers(batch.n_atoms)), int(rng.integers(3))
        e = []
        for sgn in (1, -1):
            b2 = dataclasses.replace(batch, pos=batch.pos.astype(np.float64).copy())
            b2.pos[k, a] += sgn * h
            e.append(evaluate(b2, params, nl, want_stress=False).energy_mean[0])
        fd = -(e[0] - e[1]) / (2 * h)
        assert abs(fd - r.forces[k, a]) < 1e-6 * max(1.0, abs(fd))


def test_bessel_model_energy_smooth_at_cutoff():
    """A dimer pulled through r_c: energy and force go continuously to the
    isolated-atom values (the basis and the cutoff both vanish with zero
    slope)."""
    from workloads import make_batch
    _, params, spec = _bessel_model("tiny")
    def dimer(d):
        pos = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
        b = make_batch([(pos, np.array([0, 1], np.int32), np.eye(3) * 40.0, (0, 0, 0))])
        b.pos = pos
        return evaluate(b, params, brute_force_neighbors(b, spec.r_cut))
    far = dimer(spec.r_cut + 0.5)
    near = dimer(spec.r_cut - 1e-3)
    assert abs(near.energy_mean[0] - far.energy_mean[0]) < 1e-9
    assert np.abs(near.forces).max() < 1e-6
