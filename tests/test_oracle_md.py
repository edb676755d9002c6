"""Pins of the oracle velocity-Verlet integrator: time reversibility, total
energy conservation at second order in dt, and the unit constant."""
import numpy as np

from oracle.md import velocity_verlet, kinetic_energy, ACCEL_UNIT
from workloads import make_workload


def _setup():
    b, p, s = make_workload("tiny")
    rng = np.random.default_rng(0)
    masses = np.where(b.species == 0, 6.94, 15.999)
    v = rng.normal(size=(b.n_atoms, 3)) * np.sqrt(8.617333e-5 * 300 * ACCEL_UNIT / masses)[:, None]
    return b, p, masses, v


def test_unit_constant():
    # 1 eV / (1 A * 1 amu) in A/fs^2: 1.602176634e-19 J / (1e-10 m * 1.66053906660e-27 kg) * 1e-20 (A/fs^2 per m/s^2)
    assert abs(1.602176634e-19 / (1e-10 * 1.66053906660e-27) * 1e-20 - ACCEL_UNIT) < 1e-8


def test_time_reversibility():
    b, p, m, v = _setup()
    x0 = b.pos.astype(np.float64)
    xs, vs, _ = velocity_verlet(b, p, x0, v, m, 0.5, 5)
    xb, vb, _ = velocity_verlet(b, p, xs[-1], -vs[-1], m, 0.5, 5)
    assert np.abs(xb[-1] - x0).max() < 1e-10
    assert np.abs(vb[-1] + v).max() < 1e-10


def test_energy_drift_second_order():
    b, p, m, v = _setup()
    x0 = b.pos.astype(np.float64)
    drifts = []
    for dt in (0.5, 0.25):
        n = int(round(4.0 / dt))
        xs, vs, es = velocity_verlet(b, p, x0, v, m, dt, n)
        tot = np.array([e + kinetic_energy(vv, m) for e, vv in zip(es, vs)])
        drifts.append(np.abs(tot - tot[0]).max())
    assert drifts[1] < drifts[0] / 3.0       # ~ dt^2 scaling
