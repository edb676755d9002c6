"""Pins of the oracle radial basis, moments and invariants: closed forms of
the basis and cutoff, dimer / trimer / octahedron geometries worked out by
hand, trace identities, rotation covariance of the moments and rotation
invariance of every feature."""
import math

import numpy as np
import pytest
import torch

from oracle import brute_force_neighbors, cutoff_fn, radial_basis, feature_index, invariants
from oracle.gmnn import atomic_energies, radial_functions
from workloads.configs import ModelSpec, make_params
from conftest import make_cluster

SPEC = ModelSpec(n_species=2, r_cut=5.0, hidden=(8, 8), psi_scale=0.37)


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def test_basis_centres_and_cutoff_values():
    mu = SPEC.r_min + SPEC.delta * np.arange(SPEC.n_basis)
    g = radial_basis(_t(mu), SPEC).numpy()
    assert np.allclose(np.diag(g), 1.0, atol=0, rtol=1e-15)
    # neighbouring centre: exp(-gamma delta^2) = exp(-1/2)
    assert np.allclose(g[0, 1], math.exp(-0.5), rtol=1e-14)
    fc = cutoff_fn(_t([0.0, 2.5, 5.0, 5.5]), 5.0).numpy()
    assert np.allclose(fc, [1.0, 0.5, 0.0, 0.0], atol=1e-15)
    # zero slope at r_c
    r = _t([5.0 - 1e-6]).requires_grad_(True)
    (d,) = torch.autograd.grad(cutoff_fn(r, 5.0).sum(), r)
    assert abs(float(d)) < 1e-5


def test_radial_function_zero_beyond_cutoff():
    p = make_params(SPEC, 0)
    R = radial_functions(_t([4.9, 5.0, 6.0]), torch.tensor([0, 1, 1]), torch.tensor([1, 0, 1]), _t(p.beta), SPEC)
    assert torch.all(R[1:] == 0) and torch.all(R[0] != 0)


def _psi(batch, params):
    nl = brute_force_neighbors(batch, params.spec.r_cut)
    _, G, P = atomic_energies(batch, params, nl, want_aux=True)
    return nl, G.detach().numpy(), [x.detach().numpy() for x in P]


def _R(params, zi, zj, r):
    return radial_functions(_t([r]), torch.tensor([zi]), torch.tensor([zj]), _t(params.beta), params.spec)[0].numpy()


def test_species_pair_coefficients_by_hand():
    """R_s of a pair seen from atom i uses beta[Z_i, Z_j] (Section 2.1: the
    radial functions depend on the species of the centre and of the
    neighbour, in that order).  One-hot coefficient tables on an asymmetric
    species pair, with R_s written out from exp and cos alone:
      beta[0, 1, s, k] = 1 only at (s, k) = (2, 3), beta[1, 0, s, k] = 1 only at
      (s, k) = (4, 0), every other entry zero;
      atom 0 (species 0): Psi0[0, s] = c f_c(r) exp(-gamma (r - mu_3)^2) at s = 2,
      atom 1 (species 1): Psi0[1, s] = c f_c(r) exp(-gamma (r - mu_0)^2) at s = 4,
      zero in every other channel."""
    import copy
    p = copy.deepcopy(make_params(SPEC, 3))
    p.beta = np.zeros_like(p.beta)
    p.beta[0, 1, 2, 3] = 1.0
    p.beta[1, 0, 4, 0] = 1.0
    b = make_cluster([[10, 10, 10], [10.0, 12.6, 11.1]], [0, 1])
    _, _, (P0, P1, _, _) = _psi(b, p)
    r = float(np.linalg.norm(b.pos[1].astype(np.float64) - b.pos[0]))
    delta = (5.0 - 0.5) / 6.0
    gamma = 1.0 / (2.0 * delta * delta)
    fc = 0.5 * (math.cos(math.pi * r / 5.0) + 1.0)
    want0 = np.zeros(5)
    want0[2] = 0.37 * fc * math.exp(-gamma * (r - (0.5 + 3 * delta)) ** 2)
    want1 = np.zeros(5)
    want1[4] = 0.37 * fc * math.exp(-gamma * (r - 0.5) ** 2)
    assert np.allclose(P0[0], want0, rtol=1e-13, atol=1e-300)
    assert np.allclose(P0[1], want1, rtol=1e-13, atol=1e-300)
    # the same numbers with the tables swapped move to the other atom
    p.beta = np.ascontiguousarray(p.beta.transpose(1, 0, 2, 3))
    _, _, (Q0, _, _, _) = _psi(b, p)
    h0, h1 = _hand_R(r, 2, 3, 4, 0)
    assert np.allclose(Q0[0], h0, rtol=1e-13, atol=1e-300)
    assert np.allclose(Q0[1], h1, rtol=1e-13, atol=1e-300)


def _hand_R(r, s01, k01, s10, k10):
    """Psi0 rows of the dimer for the transposed one-hot tables: atom 0 now
    sees beta[0, 1] = old beta[1, 0] (channel s10, basis k10), atom 1 sees the
    old beta[0, 1] (channel s01, basis k01)."""
    delta = (5.0 - 0.5) / 6.0
    gamma = 1.0 / (2.0 * delta * delta)
    fc = 0.5 * (math.cos(math.pi * r / 5.0) + 1.0)
    a0 = np.zeros(5)
    a0[s10] = 0.37 * fc * math.exp(-gamma * (r - (0.5 + k10 * delta)) ** 2)
    a1 = np.zeros(5)
    a1[s01] = 0.37 * fc * math.exp(-gamma * (r - (0.5 + k01 * delta)) ** 2)
    return a0, a1


def test_dimer_closed_form():
    p = make_params(SPEC, 1)
    u = np.array([0.3, -0.5, 0.8]); u /= np.linalg.norm(u)
    r = 3.1
    b = make_cluster([[10, 10, 10], list(10 + r * u)], [0, 1])
    nl, G, (P0, P1, P2, P3) = _psi(b, p)
    assert nl.n_pairs == 2
    u32 = (b.pos[1].astype(np.float64) - b.pos[0]); r32 = np.linalg.norm(u32); u32 /= r32
    R = SPEC.psi_scale * _R(p, 0, 1, r32)
    assert np.allclose(P0[0], R, rtol=1e-13)
    assert np.allclose(P1[0], R[:, None] * u32, rtol=1e-13, atol=1e-15)
    assert np.allclose(P2[0], R[:, None, None] * np.outer(u32, u32), rtol=1e-12, atol=1e-15)
    assert np.allclose(P3[0], R[:, None, None, None] * np.einsum("a,b,c->abc", u32, u32, u32), rtol=1e-12, atol=1e-15)
    # every pair invariant is R_s1 R_s2, every triple R_s1 R_s2 R_s3 (|u| = 1)
    for f, (fam, s1, s2, s3) in enumerate(feature_index(5)):
        if fam == 1:
            want = R[s1]
        elif fam in (2, 3, 4):
            want = R[s1] * R[s2]
        else:
            want = R[s1] * R[s2] * R[s3]
        assert np.isclose(G[0, f], want, rtol=1e-11, atol=1e-14), (fam, s1, s2, s3)


def test_octahedron_closed_form():
    p = make_params(SPEC, 2)
    r = 2.0
    nbr = [[r, 0, 0], [-r, 0, 0], [0, r, 0], [0, -r, 0], [0, 0, r], [0, 0, -r]]
    pos = [[10, 10, 10]] + [[10 + a, 10 + b, 10 + c] for a, b, c in nbr]
    b = make_cluster(pos, [0] + [1] * 6)
    _, G, (P0, P1, P2, P3) = _psi(b, p)
    R = SPEC.psi_scale * _R(p, 0, 1, r)
    assert np.allclose(P0[0], 6 * R, rtol=1e-13)
    assert np.allclose(P1[0], 0, atol=1e-14)
    assert np.allclose(P3[0], 0, atol=1e-14)
    assert np.allclose(P2[0], 2 * R[:, None, None] * np.eye(3), rtol=1e-13, atol=1e-14)
    # family 3: Psi2:Psi2 = 4 R R tr(I) = 12 R R; family 5: tr(8 R R R I) = 24 R R R
    for f, (fam, s1, s2, s3) in enumerate(feature_index(5)):
        if fam == 3:
            assert np.isclose(G[0, f], 12 * R[s1] * R[s2], rtol=1e-12)
        if fam == 5:
            assert np.isclose(G[0, f], 24 * R[s1] * R[s2] * R[s3], rtol=1e-12)
        if fam in (2, 4, 6, 7, 8):
            assert abs(G[0, f]) < 1e-13


@pytest.mark.parametrize("theta", [0.7, 1.9, 2.6])
def test_trimer_closed_forms(theta):
    """Centre atom with two neighbours at distances r1, r2 and angle theta:
    a_s, b_s are their radial values and u, v their directions.  Every family
    reduces to a polynomial in cos(theta) worked out by hand."""
    p = make_params(SPEC, 3)
    r1, r2 = 2.2, 3.4
    u = np.array([1.0, 0.0, 0.0]); v = np.array([math.cos(theta), math.sin(theta), 0.0])
    b = make_cluster([[10, 10, 10], list(10 + r1 * u), list(10 + r2 * v)], [0, 1, 0], box=80.0)
    nl, G, _ = _psi(b, p)
    x = b.pos.astype(np.float64)
    du, dv = x[1] - x[0], x[2] - x[0]
    # the outer atoms also see each other; only row 0 is checked
    a = _R(p, 0, 1, np.linalg.norm(du)); bb = _R(p, 0, 0, np.linalg.norm(dv))
    c = SPEC.psi_scale
    cs = float(du @ dv / np.linalg.norm(du) / np.linalg.norm(dv))
    for f, (fam, s1, s2, s3) in enumerate(feature_index(5)):
        A1, B1 = a[s1], bb[s1]
        A2, B2 = a[s2], bb[s2]
        A3, B3 = a[s3], bb[s3]
        if fam == 1:
            want = c * (A1 + B1)
        elif fam in (2, 3, 4):
            k = fam - 1
            want = c * c * (A1 * A2 + B1 * B2 + (A1 * B2 + B1 * A2) * cs ** k)
        elif fam == 5:
            mixed = A1 * A2 * B3 + A1 * B2 * A3 + B1 * A2 * A3 + A1 * B2 * B3 + B1 * A2 * B3 + B1 * B2 * A3
            want = c ** 3 * (A1 * A2 * A3 + B1 * B2 * B3 + mixed * cs ** 2)
        elif fam == 6:
            want = c ** 3 * (A3 * (A1 + B1 * cs) * (A2 + B2 * cs) + B3 * (A1 * cs + B1) * (A2 * cs + B2))
        elif fam == 7:
            pq = A2 * B3 + B2 * A3
            want = c ** 3 * (A1 * (A2 * A3 + pq * cs ** 3 + B2 * B3 * cs ** 2)
                             + B1 * (A2 * A3 * cs ** 2 + pq * cs ** 3 + B2 * B3))
        else:
            want = c ** 3 * (A2 * (A1 + B1 * cs) * (A3 + B3 * cs ** 2) + B2 * (A1 * cs + B1) * (A3 * cs ** 2 + B3))
        assert np.isclose(G[0, f], want, rtol=1e-11, atol=1e-13), (fam, s1, s2, s3, G[0, f], want)


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_trace_identities_and_rotation_covariance():
    rng = np.random.default_rng(7)
    p = make_params(SPEC, 4)
    pos = 10 + rng.random((12, 3)) * 5.0
    sp = rng.integers(0, 2, 12)
    b = make_cluster(pos, sp)
    _, G, (P0, P1, P2, P3) = _psi(b, p)
    assert np.allclose(np.einsum("nsaa->ns", P2), P0, rtol=1e-12, atol=1e-14)
    assert np.allclose(np.einsum("nsabb->nsa", P3), P1, rtol=1e-12, atol=1e-14)
    Q = _random_rotation(rng)
    pos_r = 30 + (pos - 12.5) @ Q.T
    b2 = make_cluster(pos_r, sp, box=80.0)
    _, G2, (Q0, Q1, Q2, Q3) = _psi(b2, p)
    # positions were rounded to float32 after rotation: tolerance ~1e-6
    assert np.allclose(Q1, np.einsum("ab,nsb->nsa", Q, P1), atol=2e-6)
    assert np.allclose(Q2, np.einsum("ab,cd,nsbd->nsac", Q, Q, P2), atol=2e-6)
    assert np.allclose(Q3, np.einsum("ab,cd,ef,nsbdf->nsace", Q, Q, Q, P3), atol=2e-6)
    assert np.allclose(G2, G, atol=1e-5)


def test_invariants_exactly_invariant_under_rotating_the_moments():
    rng = np.random.default_rng(9)
    S = 5
    P0 = torch.as_tensor(rng.normal(size=(3, S)))
    P1 = torch.as_tensor(rng.normal(size=(3, S, 3)))
    A = rng.normal(size=(3, S, 3, 3)); P2 = torch.as_tensor(A + A.transpose(0, 1, 3, 2))
    T = rng.normal(size=(3, S, 3, 3, 3))
    T = sum(T.transpose(0, 1, *perm) for perm in [(2, 3, 4), (2, 4, 3), (3, 2, 4), (3, 4, 2), (4, 2, 3), (4, 3, 2)])
    P3 = torch.as_tensor(T)
    G = invariants(P0, P1, P2, P3).numpy()
    assert G.shape == (3, 360)
    Q = torch.as_tensor(_random_rotation(rng))
    R1 = torch.einsum("ab,nsb->nsa", Q, P1)
    R2 = torch.einsum("ab,cd,nsbd->nsac", Q, Q, P2)
    R3 = torch.einsum("ab,cd,ef,nsbdf->nsace", Q, Q, Q, P3)
    G2 = invariants(P0, R1, R2, R3).numpy()
    assert np.allclose(G, G2, rtol=1e-11, atol=1e-11)
    # a reflection is also an orthogonal map: invariants are even in it
    Rf = torch.diag(torch.tensor([-1.0, 1.0, 1.0], dtype=torch.float64))
    G3 = invariants(P0, torch.einsum("ab,nsb->nsa", Rf, P1), torch.einsum("ab,cd,nsbd->nsac", Rf, Rf, P2),
                    torch.einsum("ab,cd,ef,nsbdf->nsace", Rf, Rf, Rf, P3)).numpy()
    assert np.allclose(G, G3, rtol=1e-12, atol=1e-12)


def test_feature_count_and_order():
    idx = feature_index(5)
    assert len(idx) == 360 == SPEC.n_features
    fams = [f[0] for f in idx]
    assert [fams.count(k) for k in range(1, 9)] == [5, 15, 15, 15, 35, 75, 75, 125]
    assert fams == sorted(fams)
