"""Pins of the oracle energies, forces, stress and head statistics: finite
differences, invariances, the supercell identity for small periodic cells,
cutoff smoothness, closed forms of the readout and shallow-ensemble
identities."""
import math

import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors, evaluate
from oracle.gmnn import atomic_energies, mlp, mlp_input_grad, swish, _bf16, split_matmul
from workloads import make_batch, make_workload
from workloads.configs import ModelSpec, make_params
from conftest import make_cluster


def _energy(batch, params, pos64=None, cell=None):
    """Total (head-mean) energy with positions given in float64, the list
    rebuilt from the float32-rounded positions but evaluated at pos64."""
    nl = brute_force_neighbors(batch, params.spec.r_cut)
    pos = None if pos64 is None else torch.as_tensor(pos64)
    E = atomic_energies(batch if cell is None else cell, params, nl, pos=pos)
    return float(E.mean(1).sum())


@pytest.fixture(scope="module")
def tiny():
    b, p, s = make_workload("tiny")
    nl = brute_force_neighbors(b, s.model.r_cut)
    return b, p, nl


def test_forces_match_central_differences(tiny):
    b, p, nl = tiny
    r = evaluate(b, p, nl)
    x0 = b.pos.astype(np.float64)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(12):
        k, a = int(rng.integers(48)), int(rng.integers(3))
        vals = []
        for s in (1, -1, 2, -2):
            x = x0.copy(); x[k, a] += s * h
            vals.append(float(atomic_energies(b, p, nl, pos=torch.as_tensor(x)).mean(1).sum()))
        d1 = (vals[0] - vals[1]) / (2 * h)
        d2 = (vals[2] - vals[3]) / (4 * h)
        fd = (4 * d1 - d2) / 3                        # Richardson: O(h^4)
        assert abs(-fd - r.forces[k, a]) < 1e-7 * max(1.0, abs(fd))


def test_net_force_zero_and_translation_invariance(tiny):
    b, p, nl = tiny
    r = evaluate(b, p, nl)
    assert np.abs(r.forces.sum(0)).max() < 1e-11
    x = b.pos.astype(np.float64) + np.array([0.37, -1.1, 2.9])
    E2 = float(atomic_energies(b, p, nl, pos=torch.as_tensor(x)).mean(1).sum())
    assert abs(E2 - r.energy_mean[0]) < 1e-10


def test_stress_matches_strain_differences(tiny):
    b, p, nl = tiny
    r = evaluate(b, p, nl)
    V = abs(np.linalg.det(b.cell[0]))
    h = 1e-6
    for (a, c) in [(0, 0), (1, 2), (2, 1), (0, 1)]:
        vals = []
        for s in (1, -1):
            eps = np.zeros((1, 3, 3)); eps[0, a, c] = s * h
            vals.append(float(atomic_energies(b, p, nl, strain=torch.as_tensor(eps)).mean(1).sum()))
        fd = (vals[0] - vals[1]) / (2 * h) / V
        assert abs(fd - r.stress[0, a, c]) < 1e-7
    assert np.allclose(r.stress[0], r.stress[0].T, atol=1e-12)


def test_supercell_energy_is_additive():
    """The 8 A box is narrower than 2 r_c (several images of one neighbour);
    its 2x2x2 supercell has the same energy density, which pins the image
    handling of the list and the sum over neighbours."""
    b, p, s = make_workload("tiny")
    e1 = evaluate(b, p, brute_force_neighbors(b, 5.0), want_stress=False).energy_mean[0]
    L = 8.0
    pos = np.concatenate([b.pos.astype(np.float64) + L * np.array(o) for o in np.ndindex(2, 2, 2)])
    sp = np.tile(b.species, 8)
    b8 = make_batch([(pos.astype(np.float32), sp, np.eye(3) * 2 * L, (1, 1, 1))])
    # evaluate at the exact float64 copies (x + 8 A is not exact in float32)
    E8 = atomic_energies(b8, p, brute_force_neighbors(b8, 5.0), pos=torch.as_tensor(pos))
    e8 = float(E8.mean(1).sum())
    assert abs(e8 - 8 * e1) < 1e-11 * abs(e8)


def _rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_rotation_and_permutation_invariance(tiny):
    b, p, nl = tiny
    r = evaluate(b, p, nl)
    rng = np.random.default_rng(3)
    Q = _rot(rng)
    # rotate positions and lattice together; evaluate at the exact (float64)
    # rotated positions with the same (i, j, S) list
    from workloads import Batch
    b_r = Batch(b.pos, b.species, b.cell @ Q.T, b.pbc, b.atom_ptr)
    x = b.pos.astype(np.float64) @ Q.T
    Er = float(atomic_energies(b_r, p, nl, pos=torch.as_tensor(x)).mean(1).sum())
    assert abs(Er - r.energy_mean[0]) < 1e-10
    perm = rng.permutation(48)
    bp = make_batch([(b.pos[perm], b.species[perm], b.cell[0], (1, 1, 1))])
    rp = evaluate(bp, p, brute_force_neighbors(bp, 5.0))
    assert abs(rp.energy_mean[0] - r.energy_mean[0]) < 1e-10
    assert np.allclose(rp.forces, r.forces[perm], atol=1e-11)


def test_energy_is_smooth_at_the_cutoff():
    """A dimer: E(r) - E(r_c) vanishes like (r_c - r)^2 as r -> r_c (the cosine
    cutoff has zero value and zero slope there) and the force is continuous."""
    spec = ModelSpec(n_species=1, r_cut=5.0, hidden=(8, 8), psi_scale=0.5)
    p = make_params(spec, 11)

    def E(r):
        b = make_cluster([[10, 10, 10], [10 + r, 10, 10]], [0, 0])
        nl = brute_force_neighbors(b, 5.0)
        return float(atomic_energies(b, p, nl, pos=torch.as_tensor([[10, 10, 10], [10 + r, 10, 10.0]])).sum())

    e_out = E(5.05)
    assert abs(E(5.0 + 1e-4) - e_out) < 1e-14          # beyond r_c: isolated atoms
    d1, d2 = 2e-2, 1e-2
    r1 = (E(5.0 - d1) - e_out) / d1 ** 2
    r2 = (E(5.0 - d2) - e_out) / d2 ** 2
    assert abs(r1 - r2) < 0.05 * abs(r2) + 1e-8


def test_readout_closed_forms():
    rng = np.random.default_rng(1)
    G = torch.as_tensor(rng.normal(size=(4, 6)))
    H = 3
    W1 = torch.zeros((6, H), dtype=torch.float64); b1 = torch.zeros(H, dtype=torch.float64)
    W2 = torch.as_tensor(rng.normal(size=(H, H))); b2 = torch.as_tensor([0.0, 1.0, -2.0], dtype=torch.float64)
    W3 = torch.as_tensor([[1.0], [2.0], [3.0]], dtype=torch.float64); b3 = torch.as_tensor([0.25], dtype=torch.float64)
    y = mlp(G, W1, b1, W2, b2, W3, b3).numpy()
    sw = lambda x: x / (1 + math.exp(-x))
    want = 1.0 * sw(0.0) + 2.0 * sw(1.0) + 3.0 * sw(-2.0) + 0.25
    assert np.allclose(y, want, rtol=1e-15)
    assert float(swish(torch.tensor(0.0, dtype=torch.float64))) == 0.0


def test_hand_written_network_backward_matches_autograd():
    rng = np.random.default_rng(2)
    t = lambda *s: torch.as_tensor(rng.normal(size=s))
    G = t(5, 7).requires_grad_(True)
    W1, b1, W2, b2, W3, b3 = t(7, 6), t(6), t(6, 4), t(4), t(4, 3), t(3)
    ybar = t(5, 3)
    y = mlp(G, W1, b1, W2, b2, W3, b3)
    (g,) = torch.autograd.grad((y * ybar).sum(), G)
    assert np.allclose(mlp_input_grad(G.detach(), W1, b1, W2, b2, W3, b3, ybar).numpy(), g.numpy(), rtol=1e-12, atol=1e-13)


def test_bf16_rounding_is_round_to_nearest_even():
    x = torch.tensor([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -(1.0 + 2.0 ** -8)],
                     dtype=torch.float64)
    assert _bf16(x).tolist() == [1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -1.0]


def test_energy_linear_in_scale_and_shift(tiny):
    b, p, nl = tiny
    e0 = evaluate(b, p, nl).energy_mean[0]
    import copy
    q = copy.deepcopy(p); q.shift = p.shift + 0.5
    e1 = evaluate(b, q, nl).energy_mean[0]
    assert abs(e1 - e0 - 0.5 * 48) < 1e-10
    q = copy.deepcopy(p); q.scale = 2 * p.scale; q.shift = 2 * p.shift
    r2 = evaluate(b, q, nl)
    assert abs(r2.energy_mean[0] - 2 * e0) < 1e-9
    assert np.allclose(r2.forces, 2 * evaluate(b, p, nl).forces, atol=1e-12)


def test_shallow_ensemble_statistics():
    b, p, s = make_workload("ensemble", n_structs=3)
    nl = brute_force_neighbors(b, 5.0)
    r = evaluate(b, p, nl, want_force_var=True)
    M = p.spec.n_heads
    assert r.energy.shape == (3, M)
    assert np.allclose(r.energy_mean, r.energy.mean(1), rtol=1e-14)
    assert np.allclose(r.energy_var, r.energy.var(1), rtol=1e-12)
    assert np.all(r.force_var >= 0)
    # mean of per-head forces equals the force of the mean (linearity); the
    # variance uses those per-head forces, so rebuild it from single heads
    import copy
    Fm = []
    for m in range(M):
        q = copy.deepcopy(p)
        q.W3 = p.W3[:, m:m + 1]; q.b3 = p.b3[m:m + 1]
        q.spec = type(p.spec)(**{**p.spec.__dict__, "n_heads": 1})
        Fm.append(evaluate(b, q, nl).forces)
    Fm = np.stack(Fm)
    assert np.allclose(Fm.mean(0), r.forces, atol=1e-11)
    assert np.allclose(((Fm - r.forces) ** 2).sum(-1).mean(0), r.force_var, rtol=1e-9, atol=1e-12)
    # identical heads: zero variance
    q = copy.deepcopy(p)
    q.W3 = np.repeat(p.W3[:, :1], M, 1); q.b3 = np.repeat(p.b3[:1], M)
    rq = evaluate(b, q, nl, want_force_var=True)
    assert np.allclose(rq.energy_var, 0, atol=1e-18) and np.allclose(rq.force_var, 0, atol=1e-20)


def test_bf16_arm_is_close_to_fp64(tiny):
    b, p, nl = tiny
    r = evaluate(b, p, nl)
    rb = evaluate(b, p, nl, bf16=True)
    rms = np.sqrt((r.forces ** 2).mean())
    assert np.sqrt(((rb.forces - r.forces) ** 2).mean()) < 0.05 * rms
    assert abs(rb.energy_mean[0] - r.energy_mean[0]) / 48 < 0.05


def test_split_bf16_product_is_exact_on_16_bit_operands():
    """Operands with at most 16 significant bits are hi + lo exactly, so the
    three-term product equals the exact product minus the dropped lo.lo term
    (hand-made values: hi and lo parts chosen directly)."""
    hi_a = torch.tensor([[1.0, -2.0, 0.75]], dtype=torch.float64)
    lo_a = torch.tensor([[2.0 ** -9, -3 * 2.0 ** -12, 2.0 ** -11]], dtype=torch.float64)
    hi_b = torch.tensor([[0.5], [1.25], [-4.0]], dtype=torch.float64)
    lo_b = torch.tensor([[-2.0 ** -10], [2.0 ** -9], [5 * 2.0 ** -10]], dtype=torch.float64)
    a, b = hi_a + lo_a, hi_b + lo_b
    got = split_matmul(a, b)
    want = hi_a @ hi_b + hi_a @ lo_b + lo_a @ hi_b
    assert torch.equal(got, want)
    assert torch.allclose(a @ b - got, lo_a @ lo_b, rtol=0, atol=1e-18)


def test_split_bf16_product_error_bound():
    """For any operands the three-term product is within about 2^-15 relative
    (per term |a_k b_k|) of the exact product: far below a single bf16
    rounding (2^-9)."""
    rng = np.random.default_rng(5)
    a = torch.as_tensor(rng.normal(size=(64, 384)))
    b = torch.as_tensor(rng.normal(size=(384, 32)) / 20.0)
    err = (split_matmul(a, b) - a @ b).abs()
    scale = a.abs() @ b.abs()
    assert (err / scale).max() < 2.0 ** -15
    plain = (_bf16(a) @ _bf16(b) - a @ b).abs()
    assert (plain / scale).max() > 2.0 ** -12
