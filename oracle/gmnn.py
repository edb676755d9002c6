"""GMNN energy, forces, stress and training gradients in float64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain PyTorch CPU ops
in float64 on full (unpacked) Cartesian tensors; derivatives come from
autograd applied to the plain definition, so they are exact up to rounding.

Method (Section 2.1 of the paper):
  * additive energy  E = sum_i E_i(G_i)                       (eq. energy_sum)
  * radial functions R_{Zi,Zj,s}(r) = f_c(r) sum_k beta[Zi,Zj,s,k] g_k(r),
    g_k equidistant Gaussians, f_c a cosine cutoff              (Section 2.1)
  * moments Psi_{i,L,s} = c_psi sum_{j != i} R_s(r_ij) rhat_ij^{(x)L}, L<=3
                                                                (eq. basis_fn)
  * invariants G_i from full tensor contractions up to L = 3 and 4-body
    terms                                                    (eq. contraction)
  * E_i = sigma_{Z_i} NN(G_i) + mu_{Z_i}                       (eq. scale_shift)
  * forces and virials as gradients w.r.t. positions and strain (Section 3.3)
  * shallow ensembles: heads share everything but the last layer; energy mean
    and population variance over heads; mean force = force of the mean energy
                                                  (Section 2.2, eq. uncertainty,
                                                   eq. jacobian, sign: F=-dE/dr)

Readings where the paper is silent (each listed in the design notes):
  * cutoff f_c(r) = (cos(pi r / r_c) + 1)/2 for r < r_c, else 0;
  * g_k(r) = exp(-gamma (r - mu_k)^2), mu_k = r_min + k*delta,
    delta = (r_c - r_min)/(K-1), gamma = 1/(2 delta^2); or the Bessel-like
    f_n of bessel_basis, with the same cutoff function;
  * the contraction set has eight families (below); the paper prints the
    first (Psi1.Psi1) and the last (Psi1 Psi3 Psi2) and elides the rest;
  * activation swish(x) = x * sigmoid(x); one network shared by all species;
  * force variance per atom: (1/M) sum_m |F_i^(m) - Fbar_i|^2.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np
import torch

DT = torch.float64


# ----------------------------------------------------------------------------
# feature order of the invariants
# ----------------------------------------------------------------------------
def feature_index(S: int):
    """List of (family, s1, s2, s3) in feature order (s unused -> -1).

    family 1: Psi0[s1]                                             s1
    family 2: Psi1[s1]_a Psi1[s2]_a                                s1<=s2
    family 3: Psi2[s1]_ab Psi2[s2]_ab                              s1<=s2
    family 4: Psi3[s1]_abc Psi3[s2]_abc                            s1<=s2
    family 5: Psi2[s1]_ab Psi2[s2]_bc Psi2[s3]_ca                  s1<=s2<=s3
    family 6: Psi1[s1]_a Psi1[s2]_b Psi2[s3]_ab                    s1<=s2, any s3
    family 7: Psi2[s1]_ab Psi3[s2]_acd Psi3[s3]_bcd                any s1, s2<=s3
    family 8: Psi1[s1]_a Psi3[s2]_abc Psi2[s3]_bc                  any s1, s2, s3
    Inside a family, tuples run in lexicographic order (last index fastest).
    """
    out = []
    r = range(S)
    out += [(1, a, -1, -1) for a in r]
    for fam in (2, 3, 4):
        out += [(fam, a, b, -1) for a in r for b in r if a <= b]
    out += [(5, a, b, c) for a in r for b in r for c in r if a <= b <= c]
    out += [(6, a, b, c) for a in r for b in r for c in r if a <= b]
    out += [(7, a, b, c) for a in r for b in r for c in r if b <= c]
    out += [(8, a, b, c) for a in r for b in r for c in r]
    return out


# ----------------------------------------------------------------------------
# pair geometry and radial functions
# ----------------------------------------------------------------------------
def pair_vectors(pos, cell, struct_of_atom, i, j, S, strain=None):
    """d_p = x_j - x_i + S_p . h_b for every pair p of structure b.
    ``strain`` ([B,3,3], zero at evaluation) deforms positions and cells of
    structure b by (I + strain_b), so dE/dstrain is the virial derivative."""
    h = cell[struct_of_atom[i]]                      # [P,3,3]
    shift = torch.einsum("pk,pkc->pc", S.to(DT), h)   # sum_k S_k h[k,:]
    d = pos[j] - pos[i] + shift
    if strain is not None:                            # strain: [B,3,3]
        d = d + torch.einsum("pab,pb->pa", strain[struct_of_atom[i]], d)
    return d


def cutoff_fn(r, r_cut):
    """Cosine cutoff (reading): (cos(pi r/r_c) + 1)/2 inside r_c, 0 outside."""
    inside = (r.real if torch.is_complex(r) else r) < r_cut
    fc = 0.5 * (torch.cos(math.pi * r / r_cut) + 1.0)
    return torch.where(inside, fc, torch.zeros_like(fc))


def radial_basis(r, spec):
    """Basis functions g_k(r), [P,K] (Section 2.1: equidistant Gaussians or
    the non-orthogonal Bessel-like functions of Kocer et al.)."""
    if getattr(spec, "basis", "gaussian") == "bessel":
        return bessel_basis(r, spec.r_cut, spec.n_basis)
    mu = spec.r_min + spec.delta * torch.arange(spec.n_basis, dtype=DT)
    return torch.exp(-spec.gamma * (r[:, None] - mu[None, :]) ** 2)


def bessel_basis(r, r_cut, K):
    """Bessel-like functions (reading; the paper names them without a
    formula): for n = 0..K-1, with x = pi r / r_c and sinc(y) = sin(y)/y,
        f_n(r) = a_n [sinc((n+1) x) + sinc((n+2) x)],
        a_n = (-1)^n sqrt(2) pi r_c^(-3/2) (n+1)(n+2) / sqrt((n+1)^2 + (n+2)^2).
    Neighbouring orders of the sine have opposite signs at r_c, so every f_n
    vanishes there with zero slope."""
    n = torch.arange(K, dtype=DT)
    a = (-1.0) ** n * math.sqrt(2.0) * math.pi * r_cut ** -1.5 * (n + 1) * (n + 2) / torch.sqrt(
        (n + 1) ** 2 + (n + 2) ** 2)
    x = (math.pi / r_cut) * r[:, None]
    y1, y2 = (n + 1) * x, (n + 2) * x
    return a * (torch.sin(y1) / y1 + torch.sin(y2) / y2)


def radial_functions(r, zi, zj, beta, spec):
    """R_{Zi,Zj,s}(r) = f_c(r) sum_k beta[Zi,Zj,s,k] g_k(r), [P,S]."""
    g = radial_basis(r, spec)
    b = beta[zi, zj]                                 # [P,S,K]
    return cutoff_fn(r, spec.r_cut)[:, None] * torch.einsum("psk,pk->ps", b, g)


# ----------------------------------------------------------------------------
# moments and invariants
# ----------------------------------------------------------------------------
def moments(d, i, zi, zj, beta, spec, n_atoms):
    """Psi_{i,L,s} for L = 0..3 as full tensors:
    Psi0 [N,S], Psi1 [N,S,3], Psi2 [N,S,3,3], Psi3 [N,S,3,3,3]."""
    r = torch.sqrt((d * d).sum(-1))
    u = d / r[:, None]
    R = radial_functions(r, zi, zj, beta, spec) * spec.psi_scale   # [P,S]
    S = spec.n_radial
    dt = d.dtype
    t0 = R
    t1 = torch.einsum("ps,pa->psa", R, u)
    t2 = torch.einsum("psa,pb->psab", t1, u)
    t3 = torch.einsum("psab,pc->psabc", t2, u)
    P0 = torch.zeros((n_atoms, S), dtype=dt).index_add(0, i, t0)
    P1 = torch.zeros((n_atoms, S, 3), dtype=dt).index_add(0, i, t1)
    P2 = torch.zeros((n_atoms, S, 3, 3), dtype=dt).index_add(0, i, t2)
    P3 = torch.zeros((n_atoms, S, 3, 3, 3), dtype=dt).index_add(0, i, t3)
    return P0, P1, P2, P3


def invariants(P0, P1, P2, P3):
    """The eight contraction families (see feature_index), [N, F]."""
    S = P0.shape[1]
    iu2 = [(a, b) for a in range(S) for b in range(S) if a <= b]
    f1 = P0
    c2 = torch.einsum("nsa,nta->nst", P1, P1)
    c3 = torch.einsum("nsab,ntab->nst", P2, P2)
    c4 = torch.einsum("nsabc,ntabc->nst", P3, P3)
    pick2 = lambda c: torch.stack([c[:, a, b] for a, b in iu2], 1)
    c5 = torch.einsum("nsab,ntbc,nuca->nstu", P2, P2, P2)
    f5 = torch.stack([c5[:, a, b, c] for a in range(S) for b in range(S) for c in range(S)
                      if a <= b <= c], 1)
    c6 = torch.einsum("nsa,ntb,nuab->nstu", P1, P1, P2)
    f6 = torch.stack([c6[:, a, b, c] for a in range(S) for b in range(S) for c in range(S)
                      if a <= b], 1)
    c7 = torch.einsum("nsab,ntacd,nubcd->nstu", P2, P3, P3)
    f7 = torch.stack([c7[:, a, b, c] for a in range(S) for b in range(S) for c in range(S)
                      if b <= c], 1)
    c8 = torch.einsum("nsa,ntabc,nubc->nstu", P1, P3, P2)
    f8 = c8.reshape(c8.shape[0], -1)
    return torch.cat([f1, pick2(c2), pick2(c3), pick2(c4), f5, f6, f7, f8], 1)


# ----------------------------------------------------------------------------
# readout
# ----------------------------------------------------------------------------
def swish(x):
    return x * torch.sigmoid(x)


def _bf16(x):
    """Round to bfloat16 (round-to-nearest-even) and widen back."""
    return x.to(torch.bfloat16).to(x.dtype)


def _bf16_parts(x):
    """High and low bfloat16 parts of x: hi = bf16(x), lo = bf16(x - hi)."""
    hi = _bf16(x)
    return hi, _bf16(x - hi)


def split_matmul(a, b):
    """a @ b from bfloat16 parts, hi_a hi_b + hi_a lo_b + lo_a hi_b: the three
    bfloat16 products of the mixed-precision arm's forward layers (the
    lo_a lo_b term, 2^-16 relative, is dropped)."""
    ah, al = _bf16_parts(a)
    bh, bl = _bf16_parts(b)
    return ah @ bh + ah @ bl + al @ bh


def _forward_z(G, W1, b1, W2, b2, bf16):
    """Pre-activations of both hidden layers.  bf16=True forms the two forward
    products from bfloat16 parts (split_matmul), as the mixed-precision GPU
    arm does."""
    mm = split_matmul if bf16 else (lambda a, b: a @ b)
    z1 = mm(G, W1) + b1
    z2 = mm(swish(z1), W2) + b2
    return z1, z2


def mlp(G, W1, b1, W2, b2, W3, b3, bf16=False):
    """NN(G) = W3^T swish(W2^T swish(W1^T G + b1) + b2) + b3, [N, heads]."""
    _, z2 = _forward_z(G, W1, b1, W2, b2, bf16)
    return swish(z2) @ W3 + b3


def mlp_input_grad(G, W1, b1, W2, b2, W3, b3, ybar, bf16=False):
    """dNN/dG contracted with ybar [N, heads], written out by hand so the
    bfloat16 arm can round the operands of the backward products (delta2,
    delta1 and the weights) to bfloat16 exactly where the GPU arm rounds them
    (its forward products are the split ones of _forward_z)."""
    rd = _bf16 if bf16 else (lambda t: t)
    z1, z2 = _forward_z(G, W1, b1, W2, b2, bf16)
    s1 = torch.sigmoid(z1)
    s2 = torch.sigmoid(z2)
    dsw1 = s1 * (1.0 + z1 * (1.0 - s1))
    dsw2 = s2 * (1.0 + z2 * (1.0 - s2))
    delta2 = dsw2 * (ybar @ W3.T)
    delta1 = dsw1 * (rd(delta2) @ rd(W2).T)
    return rd(delta1) @ rd(W1).T


# ----------------------------------------------------------------------------
# full evaluation
# ----------------------------------------------------------------------------
@dataclass
class OracleResult:
    energy: np.ndarray        # [B, heads]   per-head total energies (eV)
    energy_mean: np.ndarray   # [B]
    energy_var: np.ndarray    # [B]          population variance over heads
    atomic: np.ndarray        # [N, heads]   E_i per head
    forces: np.ndarray        # [N,3]        -dEbar/dx
    stress: np.ndarray        # [B,3,3]      (1/V) dEbar/dstrain
    force_var: np.ndarray | None   # [N]     (1/M) sum_m |F^m - Fbar|^2
    features: np.ndarray      # [N,F]
    psi: tuple                # full moment tensors (numpy)


def _tensors(batch, params, nl):
    t = lambda a, dt=DT: torch.as_tensor(np.asarray(a), dtype=dt)
    p = {k: t(v) for k, v in params.as_dict().items()}
    pos = t(batch.pos.astype(np.float64))
    cell = t(batch.cell)
    soa = torch.as_tensor(batch.struct_of_atom(), dtype=torch.long)
    sp = torch.as_tensor(batch.species, dtype=torch.long)
    i = torch.as_tensor(nl.i, dtype=torch.long)
    j = torch.as_tensor(nl.j, dtype=torch.long)
    S = torch.as_tensor(nl.S, dtype=torch.long)
    return p, pos, cell, soa, sp, i, j, S


def atomic_energies(batch, params, nl, pos=None, strain=None, bf16=False, want_aux=False, p=None):
    """E_i^(m) for every atom and head [N, heads] (autograd-traceable in pos,
    strain and the parameter tensors ``p``)."""
    spec = params.spec
    p0, pos0, cell, soa, sp, i, j, S = _tensors(batch, params, nl)
    p = p0 if p is None else p
    pos = pos0 if pos is None else pos
    d = pair_vectors(pos, cell, soa, i, j, S, strain)
    P = moments(d, i, sp[i], sp[j], p["beta"], spec, batch.n_atoms)
    G = invariants(*P)
    y = mlp(G, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"], bf16=bf16)
    E = p["scale"][sp][:, None] * y + p["shift"][sp][:, None]
    if want_aux:
        return E, G, P
    return E


def evaluate(batch, params, nl, bf16=False, want_force_var=False, want_stress=True) -> OracleResult:
    """Energies, forces, stress (and head statistics) of every structure."""
    spec = params.spec
    M = spec.n_heads
    p, pos0, cell, soa, sp, i, j, S = _tensors(batch, params, nl)
    B = batch.n_structs
    pos = pos0.clone().requires_grad_(True)
    strain = torch.zeros((B, 3, 3), dtype=DT, requires_grad=True)
    d = pair_vectors(pos, cell, soa, i, j, S, strain)
    P = moments(d, i, sp[i], sp[j], p["beta"], spec, batch.n_atoms)
    G = invariants(*P)
    y = mlp(G, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"], bf16=bf16)
    Ei = p["scale"][sp][:, None] * y + p["shift"][sp][:, None]          # [N,M]
    Eb = torch.zeros((B, M), dtype=DT).index_add(0, soa, Ei)            # [B,M]
    Ebar = Eb.mean(1)
    if bf16:
        # the bf16 arm rounds the backward operands too: take dE/dG from the
        # hand-written network backward, then autograd from G to positions
        ybar = (p["scale"][sp][:, None] / M).expand(-1, M)
        Gbar = mlp_input_grad(G.detach(), p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"], ybar, bf16=True)
        gpos, gstrain = torch.autograd.grad(G, (pos, strain), Gbar, retain_graph=want_force_var)
    else:
        gpos, gstrain = torch.autograd.grad(Ebar.sum(), (pos, strain), retain_graph=want_force_var)
    forces = -gpos
    vol = torch.abs(torch.linalg.det(cell))
    stress = gstrain / vol[:, None, None]
    fvar = None
    if want_force_var:
        Fm = []
        for m in range(M):
            if bf16:
                ybar = torch.zeros((batch.n_atoms, M), dtype=DT)
                ybar[:, m] = p["scale"][sp]
                Gbar = mlp_input_grad(G.detach(), p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"], ybar, bf16=True)
                (g,) = torch.autograd.grad(G, (pos,), Gbar, retain_graph=True)
            else:
                (g,) = torch.autograd.grad(Eb[:, m].sum(), (pos,), retain_graph=True)
            Fm.append(-g)
        Fm = torch.stack(Fm)                                             # [M,N,3]
        fvar = ((Fm - forces[None]) ** 2).sum(-1).mean(0).detach().numpy()
    var = ((Eb - Ebar[:, None]) ** 2).mean(1)
    return OracleResult(
        energy=Eb.detach().numpy(), energy_mean=Ebar.detach().numpy(), energy_var=var.detach().numpy(),
        atomic=Ei.detach().numpy(), forces=forces.detach().numpy(), stress=stress.detach().numpy(),
        force_var=fvar, features=G.detach().numpy(), psi=tuple(x.detach().numpy() for x in P))


# ----------------------------------------------------------------------------
# uncertainty-driven bias (Section 2.3, eq. udd)
# ----------------------------------------------------------------------------
def udd_bias(energy_heads, n_atoms, A, B):
    """E_bias = A [exp(-var / (M N B^2)) - 1] per structure, with var the
    population variance over the M heads of the structure's energy."""
    M = energy_heads.shape[-1]
    var = ((energy_heads - energy_heads.mean(-1, keepdim=True)) ** 2).mean(-1)
    return A * (torch.exp(-var / (M * n_atoms * B * B)) - 1.0)


@dataclass
class UddResult:
    energy: np.ndarray        # [B, heads]   unbiased per-head energies
    bias_energy: np.ndarray   # [B]
    forces: np.ndarray        # [N,3]   -d(Ebar + E_bias)/dx
    stress: np.ndarray        # [B,3,3] (1/V) d(Ebar + E_bias)/dstrain


def evaluate_udd(batch, params, nl, A, B) -> UddResult:
    """Energies, bias energy, and forces and stress of Ebar + E_bias
    (autograd through the plain definition)."""
    spec = params.spec
    M = spec.n_heads
    p, pos0, cell, soa, sp, i, j, S = _tensors(batch, params, nl)
    nb = torch.as_tensor(np.diff(batch.atom_ptr), dtype=DT)
    pos = pos0.clone().requires_grad_(True)
    strain = torch.zeros((batch.n_structs, 3, 3), dtype=DT, requires_grad=True)
    d = pair_vectors(pos, cell, soa, i, j, S, strain)
    G = invariants(*moments(d, i, sp[i], sp[j], p["beta"], spec, batch.n_atoms))
    y = mlp(G, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"])
    Ei = p["scale"][sp][:, None] * y + p["shift"][sp][:, None]
    Eb = torch.zeros((batch.n_structs, M), dtype=DT).index_add(0, soa, Ei)
    Ebias = udd_bias(Eb, nb, A, B)
    total = (Eb.mean(1) + Ebias).sum()
    gpos, gstrain = torch.autograd.grad(total, (pos, strain))
    vol = torch.abs(torch.linalg.det(cell))
    return UddResult(Eb.detach().numpy(), Ebias.detach().numpy(), (-gpos).numpy(),
                     (gstrain / vol[:, None, None]).numpy())


# ----------------------------------------------------------------------------
# training loss and parameter gradients (Section 3.4: weighted sum of loss
# terms, optionally divided by the number of atoms)
# ----------------------------------------------------------------------------
PARAM_NAMES = ("beta", "W1", "b1", "W2", "b2", "W3", "b3", "scale", "shift")


def loss_and_param_grads(batch, params, nl, E_ref, F_ref, w_E=1.0, w_F=1.0, want_pos=False):
    """L = w_E/B sum_b ((Ebar_b - E_ref_b)/N_b)^2 + w_F/(3N) sum |F - F_ref|^2
    and dL/dtheta for every parameter array (dict of numpy arrays), plus
    dL/dE_b and dL/dF (the upstream gradients a caller feeds to a backward);
    with want_pos also dL/dx [N, 3], the loss's gradient in the positions
    (through the energies and, with forces = -dE/dx, their second
    derivatives)."""
    p, pos0, cell, soa, sp, i, j, S = _tensors(batch, params, nl)
    p = {k: v.clone().requires_grad_(True) for k, v in p.items()}
    spec = params.spec
    B, N, M = batch.n_structs, batch.n_atoms, spec.n_heads
    pos = pos0.clone().requires_grad_(True)
    d = pair_vectors(pos, cell, soa, i, j, S)
    P = moments(d, i, sp[i], sp[j], p["beta"], spec, N)
    G = invariants(*P)
    y = mlp(G, p["W1"], p["b1"], p["W2"], p["b2"], p["W3"], p["b3"])
    Ei = p["scale"][sp][:, None] * y + p["shift"][sp][:, None]
    Ebar = torch.zeros((B, M), dtype=DT).index_add(0, soa, Ei).mean(1)
    (gpos,) = torch.autograd.grad(Ebar.sum(), (pos,), create_graph=True)
    F = -gpos
    nb = torch.as_tensor(np.diff(batch.atom_ptr), dtype=DT)
    Er = torch.as_tensor(E_ref, dtype=DT)
    Fr = torch.as_tensor(F_ref, dtype=DT)
    L = w_E / B * (((Ebar - Er) / nb) ** 2).sum() + w_F / (3 * N) * ((F - Fr) ** 2).sum()
    grads = torch.autograd.grad(L, [p[k] for k in PARAM_NAMES] + [Ebar, F, pos], allow_unused=True)
    out = {k: (g.detach().numpy() if g is not None else np.zeros(p[k].shape)) for k, g in zip(PARAM_NAMES, grads)}
    dLdE = grads[len(PARAM_NAMES)].detach().numpy()
    dLdF = grads[len(PARAM_NAMES) + 1].detach().numpy()
    if want_pos:
        return float(L.detach()), out, dLdE, dLdF, grads[len(PARAM_NAMES) + 2].detach().numpy()
    return float(L.detach()), out, dLdE, dLdF
