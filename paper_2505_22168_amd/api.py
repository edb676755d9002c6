"""Python binding of the GMNN library: device buffers are torch tensors, every
step of the energy/force path runs in the HIP kernels of libgmnn.so.

The binding only marshals arguments: it allocates torch tensors for the
caller-owned buffers of the C ABI, passes their device pointers and the
current torch stream, and checks the returned status.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi as A


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_device(device):
    device = torch.device(device)
    if device.type != "cuda":
        raise RuntimeError("the GMNN library runs on a HIP device only (no CPU fallback)")
    return device


# ---------------------------------------------------------------------------
class System:
    """A ragged batch of periodic structures on the device (gmnn_system)."""

    def __init__(self, pos, species, cell, pbc, atom_ptr, device="cuda"):
        device = _require_device(device)
        self.atom_ptr_host = np.ascontiguousarray(np.asarray(atom_ptr, dtype=np.int64))
        self.cell_host = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(-1, 3, 3))
        self.pbc_host = np.ascontiguousarray(np.asarray(pbc, dtype=np.uint8).reshape(-1, 3))
        self.pos = torch.as_tensor(np.asarray(pos, dtype=np.float32)).reshape(-1, 3).contiguous().to(device)
        self.species = torch.as_tensor(np.asarray(species, dtype=np.int32)).contiguous().to(device)
        self.cell = torch.as_tensor(self.cell_host).to(device)
        self.pbc = torch.as_tensor(self.pbc_host).to(device)
        self.atom_ptr = torch.as_tensor(self.atom_ptr_host).to(device)
        self.device = device

    @classmethod
    def from_batch(cls, batch, device="cuda"):
        return cls(batch.pos, batch.species, batch.cell, batch.pbc, batch.atom_ptr, device)

    @property
    def n_atoms(self):
        return int(self.atom_ptr_host[-1])

    @property
    def n_structs(self):
        return int(self.cell_host.shape[0])

    def c(self, pos=None):
        p = self.pos if pos is None else pos
        return A.gmnn_system(
            self.n_structs, self.n_atoms, _ptr(self.atom_ptr), self.atom_ptr_host.ctypes.data_as(C.c_void_p),
            _ptr(p), _ptr(self.species), _ptr(self.cell), self.cell_host.ctypes.data_as(C.c_void_p),
            _ptr(self.pbc), self.pbc_host.ctypes.data_as(C.c_void_p))


# ---------------------------------------------------------------------------
class NeighborList:
    """Device CSR neighbour list (gmnn_neighbors), canonical order."""

    def __init__(self, n_atoms: int, capacity: int, device):
        self.capacity = int(capacity)
        self.row_ptr = torch.zeros(n_atoms + 1, dtype=torch.int64, device=device)
        self.j = torch.zeros(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.shift = torch.zeros(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.rev = torch.zeros(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.atom_struct = torch.zeros(max(n_atoms, 1), dtype=torch.int32, device=device)
        self.n_pairs_dev = torch.zeros(1, dtype=torch.int64, device=device)
        self.status_dev = torch.zeros(1, dtype=torch.int32, device=device)
        self.cutoff = 0.0

    def c(self):
        return A.gmnn_neighbors(self.capacity, _ptr(self.row_ptr), _ptr(self.j), _ptr(self.shift), _ptr(self.rev),
                                _ptr(self.atom_struct), _ptr(self.n_pairs_dev), _ptr(self.status_dev),
                                C.c_float(self.cutoff))

    @property
    def n_pairs(self) -> int:
        return int(self.n_pairs_dev.item())

    @property
    def status(self) -> int:
        return int(self.status_dev.item()) & 0xFFFFFFFF

    def shifts(self):
        """Unpacked image vectors [P,3] (int64) of the first n_pairs pairs."""
        s = self.shift[: self.n_pairs].to(torch.int64)
        out = torch.stack([(s >> (8 * k)) & 0xFF for k in range(3)], 1)
        return torch.where(out >= 128, out - 256, out)

    def rows(self):
        """Centre atom of every pair [P] (int64)."""
        counts = torch.diff(self.row_ptr)
        return torch.repeat_interleave(torch.arange(len(counts), device=counts.device), counts)


def estimate_capacity(system: System, cutoff: float, skin: float) -> int:
    rl = cutoff + skin
    total = 0.0
    for b in range(system.n_structs):
        n = system.atom_ptr_host[b + 1] - system.atom_ptr_host[b]
        vol = abs(np.linalg.det(system.cell_host[b]))
        total += n * (n / vol * 4.0 / 3.0 * math.pi * rl ** 3)
    return int(total * 1.25) + 1024


def build_neighbors(system: System, cutoff: float, skin: float = 0.0, capacity: int | None = None,
                    nl: NeighborList | None = None, workspace: torch.Tensor | None = None) -> NeighborList:
    """Build the list; grows the capacity (and rebuilds) when it is too small."""
    lib = A.load()
    sysc = system.c()
    nbytes = lib.gmnn_neighbors_workspace_bytes(C.byref(sysc), cutoff, skin)
    if nbytes == 0:
        raise A.GMNNError(A.GMNN_ERR_INVALID_ARG, "gmnn_neighbors_workspace_bytes")
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=system.device)
    if nl is None:
        cap = capacity if capacity is not None else estimate_capacity(system, cutoff, skin)
        nl = NeighborList(system.n_atoms, cap, system.device)
    for _ in range(2):
        nlc = nl.c()
        st = lib.gmnn_build_neighbors(C.byref(sysc), cutoff, skin, C.byref(nlc), A.GMNN_SYNC, _ptr(workspace),
                                      nbytes, _stream())
        nl.cutoff = float(np.float32(cutoff) + np.float32(skin))
        if st == A.GMNN_ERR_CAPACITY:
            need = nl.n_pairs
            nl = NeighborList(system.n_atoms, int(need * 1.1) + 1024, system.device)
            continue
        A.check(st, "gmnn_build_neighbors")
        return nl
    raise A.GMNNError(A.GMNN_ERR_CAPACITY, "gmnn_build_neighbors")


# ---------------------------------------------------------------------------
PARAM_NAMES = ("beta", "W1", "b1", "W2", "b2", "W3", "b3", "scale", "shift")


class Model:
    """GMNN parameters on the device plus their MFMA-ordered packed copies."""

    def __init__(self, spec, params: dict, device="cuda"):
        device = _require_device(device)
        self.train_precision = "fp32"  # network precision of EnergyForcesFunction ("fp32" or "bf16")
        self.spec = spec
        self.device = device
        self.tensors = {k: torch.as_tensor(np.asarray(params[k], dtype=np.float32)).contiguous().to(device)
                        for k in PARAM_NAMES}
        lib = A.load()
        c = self._c(None)
        nbytes = lib.gmnn_model_packed_bytes(C.byref(c))
        self.packed = torch.zeros(nbytes, dtype=torch.uint8, device=device)
        self.prepare()

    @classmethod
    def from_params(cls, params, device="cuda"):
        return cls(params.spec, params.as_dict(), device)

    def _c(self, packed):
        s = self.spec
        t = self.tensors
        H1, H2 = s.hidden
        basis = {"gaussian": A.GMNN_BASIS_GAUSSIAN, "bessel": A.GMNN_BASIS_BESSEL}[getattr(s, "basis", "gaussian")]
        return A.gmnn_model(s.n_species, s.n_radial, s.n_basis, H1, H2, s.n_heads, s.r_min, s.r_cut, s.gamma,
                            s.psi_scale, *[_ptr(t[k]) for k in PARAM_NAMES], _ptr(packed), basis)

    def c(self):
        return self._c(self.packed)

    def params(self):
        """The FP32 parameter tensors in C-ABI order (beta, W1, b1, W2, b2, W3, b3, scale, shift)."""
        return [self.tensors[k] for k in PARAM_NAMES]

    # parameters the packed buffer copies (beta, scale and shift are read live)
    _PACKED = ("W1", "b1", "W2", "b2", "W3", "b3")

    def _versions(self):
        return tuple(self.tensors[k]._version for k in self._PACKED)

    def prepare(self):
        """Refresh the packed weights after the FP32 parameters changed."""
        c = self.c()
        A.check(A.load().gmnn_model_prepare(C.byref(c), _stream()), "gmnn_model_prepare")
        self._packed_versions = self._versions()

    def ensure_packed(self):
        """Re-pack if any packed parameter was modified in place since the
        last prepare() (e.g. by an optimiser step on params())."""
        if self._versions() != self._packed_versions:
            self.prepare()


@dataclass
class Outputs:
    energy: torch.Tensor        # [B, heads] float64
    forces: torch.Tensor        # [N, 3] float32
    stress: torch.Tensor | None
    energy_var: torch.Tensor | None
    force_var: torch.Tensor | None
    atomic_energy: torch.Tensor
    energy_mean: torch.Tensor     # [B] float64, mean over heads
    status: torch.Tensor          # [1] int32 device status word (GMNN_FLAG_* bits)
    bias_energy: torch.Tensor | None = None  # [B] float64 uncertainty-driven bias (udd=)
    forces_heads: torch.Tensor | None = None  # [heads, N, 3] float32 per-head forces (force_var=True)


class EnergyForces:
    """Reusable evaluator: owns the outputs and the workspace of one system /
    list / model shape, so repeated calls allocate nothing."""

    def __init__(self, model: Model, system: System, nl: NeighborList, precision: str = "bf16",
                 stress: bool = True, force_var: bool = False, plan=None, udd=None):
        """plan: None (the library's built-in choice), "auto" (the autotuned
        plan of this shape class, cached; tunes on first use), or a dict /
        tuple (schedule, lanes_per_atom[, readout[, tile_atoms]]) with
        GMNN_SCHEDULE_*, 8/16/32/64, GMNN_READOUT_* and 8/16 (0 = built-in
        choice).  udd: (A, B) for the uncertainty-driven bias
        (gmnn_energy_forces_udd; forces of Ebar + E_bias, bias energies in
        out.bias_energy; plan None or a split plan)."""
        self.model, self.system, self.nl = model, system, nl
        self.flags = (A.GMNN_PREC_BF16 if precision == "bf16" else A.GMNN_PREC_FP32)
        if precision not in ("bf16", "fp32"):
            raise ValueError(precision)
        if stress:
            self.flags |= A.GMNN_WANT_STRESS
        if force_var:
            self.flags |= A.GMNN_WANT_FORCE_VAR
        dev = system.device
        B, N, M = system.n_structs, system.n_atoms, model.spec.n_heads
        self.out = Outputs(
            energy=torch.zeros((B, M), dtype=torch.float64, device=dev),
            forces=torch.zeros((max(N, 1), 3), dtype=torch.float32, device=dev),
            stress=torch.zeros((B, 3, 3), dtype=torch.float64, device=dev) if stress else None,
            energy_var=torch.zeros(B, dtype=torch.float64, device=dev),
            force_var=torch.zeros(max(N, 1), dtype=torch.float32, device=dev) if force_var else None,
            atomic_energy=torch.zeros((max(N, 1), M), dtype=torch.float32, device=dev),
            energy_mean=torch.zeros(B, dtype=torch.float64, device=dev),
            status=torch.zeros(1, dtype=torch.int32, device=dev),
            forces_heads=torch.zeros((M, max(N, 1), 3), dtype=torch.float32, device=dev) if force_var else None)
        lib = A.load()
        self._mc = model.c()
        self._sc = system.c()
        self._nc = nl.c()
        nbytes = lib.gmnn_workspace_bytes(A.GMNN_OP_ENERGY_FORCES, C.byref(self._mc), C.byref(self._sc),
                                          C.byref(self._nc), self.flags)
        self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        self.ws_bytes = nbytes
        o = self.out
        self._oc = A.gmnn_outputs(_ptr(o.energy), _ptr(o.forces), _ptr(o.stress), _ptr(o.energy_var),
                                  _ptr(o.force_var), _ptr(o.atomic_energy), _ptr(o.energy_mean), _ptr(o.status),
                                  _ptr(o.forces_heads))
        self._plan = None
        self._udd = None
        if udd is not None:
            if isinstance(plan, str):
                raise ValueError("the biased evaluation takes None or an explicit split plan")
            self.out.bias_energy = torch.zeros(B, dtype=torch.float64, device=dev)
            self._udd = A.gmnn_udd(float(udd[0]), float(udd[1]), _ptr(self.out.bias_energy))
        self.set_plan(plan)

    def set_plan(self, plan):
        if isinstance(plan, str):
            if plan != "auto":
                raise ValueError(plan)
            from .autotune import tuned_plan
            plan = tuned_plan(self)
        if plan is None:
            self._plan = None
            return
        self._plan = A.gmnn_plan.of(plan)
        A.check(A.load().gmnn_resolve_plan(C.byref(self._mc), C.byref(self._sc), self.flags,
                                           C.byref(self._plan), None), "gmnn_resolve_plan")

    @property
    def plan(self) -> dict:
        """The plan the library runs (zero fields resolved)."""
        r = A.gmnn_plan()
        A.check(A.load().gmnn_resolve_plan(C.byref(self._mc), C.byref(self._sc), self.flags,
                                           None if self._plan is None else C.byref(self._plan), C.byref(r)),
                "gmnn_resolve_plan")
        return r.as_dict()

    def capture(self, n_evals: int = 1):
        """Capture n_evals evaluations into a HIP graph (replayed by replay())."""
        self.release()
        torch.cuda.synchronize()
        h = C.c_void_p()
        A.check(A.load().gmnn_energy_forces_graph_create(
            C.byref(self._mc), C.byref(self._sc), C.byref(self._nc), self.flags,
            None if self._plan is None else C.byref(self._plan), C.byref(self._oc), _ptr(self.workspace),
            self.ws_bytes, n_evals, C.byref(h)), "gmnn_energy_forces_graph_create")
        self._graph, self.graph_evals = h, n_evals
        return self

    def replay(self, times: int = 1) -> Outputs:
        """Launch the captured graph `times` times on the current stream."""
        if getattr(self, "_graph", None) is None:
            raise RuntimeError("capture() first")
        for _ in range(times):
            A.check(A.load().gmnn_graph_launch(self._graph, _stream()), "gmnn_graph_launch")
        return self.out

    def release(self):
        if getattr(self, "_graph", None) is not None:
            A.load().gmnn_graph_destroy(self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def __call__(self, sync: bool = False) -> Outputs:
        flags = self.flags | (A.GMNN_SYNC if sync else 0)
        plan = None if self._plan is None else C.byref(self._plan)
        if self._udd is not None:
            st = A.load().gmnn_energy_forces_udd(C.byref(self._mc), C.byref(self._sc), C.byref(self._nc), flags,
                                                 plan, C.byref(self._udd), C.byref(self._oc), _ptr(self.workspace),
                                                 self.ws_bytes, _stream())
            A.check(st, "gmnn_energy_forces_udd")
            return self.out
        st = A.load().gmnn_energy_forces_plan(C.byref(self._mc), C.byref(self._sc), C.byref(self._nc), flags,
                                              plan, C.byref(self._oc), _ptr(self.workspace), self.ws_bytes,
                                              _stream())
        A.check(st, "gmnn_energy_forces")
        return self.out


def energy_forces(model: Model, system: System, nl: NeighborList, precision: str = "bf16", stress: bool = True,
                  force_var: bool = False, plan=None) -> Outputs:
    """One evaluation (allocates its outputs and workspace)."""
    return EnergyForces(model, system, nl, precision, stress, force_var, plan)(sync=False)


# ---------------------------------------------------------------------------
KB_EV_PER_K = 8.617333262e-5
ACCEL_UNIT = 9.648533e-3          # (eV/A)/amu -> A/fs^2


class MD:
    """NVE velocity-Verlet MD on the device (gmnn_md_*), with the steps
    replayed from a HIP graph.  Positions in `system.pos` are updated in place."""

    def __init__(self, model: Model, system: System, masses, dt: float, skin: float, velocities=None,
                 precision: str = "fp32", capacity: int | None = None, udd=None, var_every: int = 0):
        """udd: (A, B) of the uncertainty-driven bias (bias energies in
        self.bias_energy); var_every > 0: the per-head force variance
        (self.force_var) on every var_every-th step of a call or graph, the
        head-mean forces on the others."""
        lib = A.load()
        dev = system.device
        N, B, M = system.n_atoms, system.n_structs, model.spec.n_heads
        self.model, self.system, self.lib = model, system, lib
        self.flags = A.GMNN_PREC_BF16 if precision == "bf16" else A.GMNN_PREC_FP32
        if var_every > 0:
            self.flags |= A.GMNN_WANT_FORCE_VAR
        cap = capacity if capacity is not None else int(estimate_capacity(system, model.spec.r_cut, skin) * 1.3)
        self.nl = NeighborList(N, cap, dev)
        self.nl.cutoff = float(np.float32(model.spec.r_cut) + np.float32(skin))
        self.inv_mass = (1.0 / torch.as_tensor(np.asarray(masses, dtype=np.float64))).to(torch.float32).to(dev)
        self.vel = torch.zeros((max(N, 1), 3), dtype=torch.float32, device=dev)
        if velocities is not None:
            self.vel[:N] = torch.as_tensor(np.asarray(velocities, dtype=np.float32)).to(dev)
        self.forces = torch.zeros((max(N, 1), 3), dtype=torch.float32, device=dev)
        self.energy = torch.zeros((B, M), dtype=torch.float64, device=dev)
        self.ref_pos = torch.zeros((max(N, 1), 3), dtype=torch.float32, device=dev)
        self.disp = torch.zeros(1, dtype=torch.int32, device=dev)
        self.force_var = torch.zeros(max(N, 1), dtype=torch.float32, device=dev)
        self.energy_var = torch.zeros(B, dtype=torch.float64, device=dev)
        self.bias_energy = torch.zeros(B, dtype=torch.float64, device=dev)
        self._udd = None if udd is None else A.gmnn_udd(float(udd[0]), float(udd[1]), _ptr(self.bias_energy))
        self._md = A.gmnn_md(dt, skin, _ptr(self.inv_mass), _ptr(self.vel), _ptr(self.forces), _ptr(self.energy),
                             _ptr(self.ref_pos), _ptr(self.disp),
                             None if self._udd is None else C.cast(C.pointer(self._udd), C.c_void_p),
                             int(var_every), _ptr(self.force_var), _ptr(self.energy_var))
        self._mc, self._sc, self._nc = model.c(), system.c(), self.nl.c()
        nbytes = lib.gmnn_md_workspace_bytes(C.byref(self._mc), C.byref(self._sc), C.byref(self._nc), self.flags)
        if nbytes == 0:
            raise A.GMNNError(A.GMNN_ERR_INVALID_ARG, "gmnn_md_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.ws_bytes = nbytes
        self.graph = None
        self.graph_steps = 0
        A.check(lib.gmnn_md_init(C.byref(self._mc), C.byref(self._sc), C.byref(self._nc), C.byref(self._md),
                                 self.flags, _ptr(self.workspace), nbytes, _stream()), "gmnn_md_init")

    def steps(self, n: int):
        """n steps launched eagerly (one C call, no host synchronisation)."""
        A.check(self.lib.gmnn_md_steps(C.byref(self._mc), C.byref(self._sc), C.byref(self._nc), C.byref(self._md),
                                       self.flags, n, _ptr(self.workspace), self.ws_bytes, _stream()),
                "gmnn_md_steps")

    def capture(self, n: int):
        """Capture n steps into a HIP graph (replayed by run())."""
        self.release()
        torch.cuda.synchronize()
        h = C.c_void_p()
        A.check(self.lib.gmnn_md_graph_create(C.byref(self._mc), C.byref(self._sc), C.byref(self._nc),
                                              C.byref(self._md), self.flags, n, _ptr(self.workspace), self.ws_bytes,
                                              C.byref(h)), "gmnn_md_graph_create")
        self.graph, self.graph_steps = h, n

    def run(self, replays: int = 1):
        for _ in range(replays):
            A.check(self.lib.gmnn_md_graph_launch(self.graph, _stream()), "gmnn_md_graph_launch")

    def release(self):
        if self.graph is not None:
            self.lib.gmnn_md_graph_destroy(self.graph)
            self.graph = None

    def status(self) -> int:
        return self.nl.status

    def kinetic_energy(self, masses) -> float:
        """FP64 kinetic energy in eV (diagnostic, computed on the host)."""
        v = self.vel[: self.system.n_atoms].double().cpu().numpy()
        return float(0.5 * (np.asarray(masses)[:, None] * v * v).sum() / ACCEL_UNIT)

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def maxwell_boltzmann(masses, temperature: float, seed: int):
    """Velocities (A/fs) at `temperature` (K) with zero total momentum."""
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, dtype=np.float64)
    sig = np.sqrt(KB_EV_PER_K * temperature * ACCEL_UNIT / m)
    v = rng.normal(size=(len(m), 3)) * sig[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    return v.astype(np.float32)


# ---------------------------------------------------------------------------
def param_grads(model: Model, system: System, nl: NeighborList, dL_dE, dL_dF, workspace=None,
                precision: str = "fp32", out=None, lanes16: bool = False, per_head: bool = False,
                dL_dpos=None):
    """Gradients of a loss w.r.t. every model parameter (gmnn_backward), given
    dL/dE per structure (head-mean energy, float64 [B]) and dL/dF [N,3];
    precision "bf16" runs the network products of the double backward in BF16
    and the weight-gradient products as three BF16 products of split FP32
    operands (about 16 significant bits per product).  per_head: the
    upstream gradients are per head, dL/dE^m [B, heads] and dL/dF^m
    [heads, N, 3] (shallow-ensemble losses; one double backward per head).
    dL_dpos: an FP32 device tensor [N, 3] that receives the loss's gradient
    in the positions (may be None).

    `out` (a dict of FP32 device tensors shaped like model.tensors) receives
    the gradients; the call overwrites every element, so neither `out` nor a
    freshly allocated result needs clearing first."""
    if precision not in ("fp32", "bf16"):
        raise ValueError(precision)
    flags = ((A.GMNN_PREC_BF16 if precision == "bf16" else 0) | (A.GMNN_BACKWARD_LANES16 if lanes16 else 0)
             | (A.GMNN_BACKWARD_PER_HEAD if per_head else 0))
    lib = A.load()
    dev = system.device
    B, N, M = system.n_structs, system.n_atoms, model.spec.n_heads
    dE = torch.as_tensor(dL_dE, dtype=torch.float64, device=dev).contiguous()
    dF = torch.as_tensor(dL_dF, dtype=torch.float32, device=dev).contiguous()
    if per_head:
        dF = dF.reshape(M, -1, 3)
        if dE.shape != (B, M) or dF.shape[1] < N:
            raise ValueError(f"per-head gradients need dL_dE [{B}, {M}] and dL_dF [{M}, {N}, 3]")
        if dF.shape[1] != N:
            dF = dF[:, :N].contiguous()  # the library reads head m's rows at m * 3N
    else:
        dF = dF.reshape(-1, 3)
    if out is None:
        grads = {k: torch.empty_like(v) for k, v in model.tensors.items()}
    else:
        grads = out
        for k, v in model.tensors.items():
            g = grads[k]
            if g.shape != v.shape or g.dtype != torch.float32 or g.device != v.device or not g.is_contiguous():
                raise ValueError(f"out[{k!r}] must be a contiguous float32 tensor of shape {tuple(v.shape)} on {v.device}")
    gc = A.gmnn_param_grads(*[_ptr(grads[k]) for k in PARAM_NAMES])
    model.ensure_packed()
    mc, sc, nc = model.c(), system.c(), nl.c()
    nbytes = lib.gmnn_workspace_bytes(A.GMNN_OP_BACKWARD, C.byref(mc), C.byref(sc), C.byref(nc), flags)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    if dL_dpos is not None and (dL_dpos.dtype != torch.float32 or not dL_dpos.is_contiguous()
                                or dL_dpos.numel() < 3 * N or dL_dpos.device.type != "cuda"):
        raise ValueError(f"dL_dpos must be a contiguous float32 device tensor of at least [{N}, 3]")
    st = lib.gmnn_backward(C.byref(mc), C.byref(sc), C.byref(nc), _ptr(dE), _ptr(dF), flags, C.byref(gc),
                           None if dL_dpos is None else _ptr(dL_dpos), _ptr(workspace), nbytes, _stream())
    A.check(st, "gmnn_backward")
    return grads


class EnergyForcesFunction(torch.autograd.Function):
    """(E, F) = GMNN(theta) as a differentiable torch op: forward runs
    gmnn_energy_forces, backward runs gmnn_backward (network products in
    model.train_precision, "fp32" or "bf16"), giving the gradients of any
    loss of E and F w.r.t. the parameter tensors.

        E, F = EnergyForcesFunction.apply(model, system, nl, *model.params())
    """

    @staticmethod
    def forward(ctx, model, system, nl, *params):
        own = model.params()
        if len(params) != len(own) or any(p is not q for p, q in zip(params, own)):
            raise ValueError("EnergyForcesFunction takes the model's own parameter tensors (model.params())")
        model.ensure_packed()  # an in-place optimiser step since the last call
        out = energy_forces(model, system, nl, precision=model.train_precision, stress=False)
        ctx.model, ctx.system, ctx.nl = model, system, nl
        return out.energy_mean.clone(), out.forces[: system.n_atoms].clone()

    @staticmethod
    def backward(ctx, gE, gF):
        B, N = ctx.system.n_structs, ctx.system.n_atoms
        gE = torch.zeros(B, dtype=torch.float64, device=ctx.system.device) if gE is None else gE.double()
        gF = torch.zeros((N, 3), dtype=torch.float32, device=ctx.system.device) if gF is None else gF.float()
        grads = param_grads(ctx.model, ctx.system, ctx.nl, gE, gF, precision=ctx.model.train_precision)
        return (None, None, None, *[grads[k] for k in PARAM_NAMES])


# ---------------------------------------------------------------------------
# batch active learning (gmnn_last_layer_features, gmnn_select_max_distance)
def last_layer_features(model: Model, system: System, nl: NeighborList, precision: str = "fp32") -> torch.Tensor:
    """Last-layer gradient features [B, H2 + 1] (float64, device) of every
    structure: the gradient of its head-mean energy w.r.t. one head's
    last-layer weights and bias."""
    if precision not in ("fp32", "bf16"):
        raise ValueError(precision)
    flags = A.GMNN_PREC_BF16 if precision == "bf16" else A.GMNN_PREC_FP32
    lib = A.load()
    model.ensure_packed()
    mc, sc, nc = model.c(), system.c(), nl.c()
    nbytes = lib.gmnn_workspace_bytes(A.GMNN_OP_FEATURES, C.byref(mc), C.byref(sc), C.byref(nc), flags)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=system.device)
    phi = torch.empty((system.n_structs, model.spec.hidden[1] + 1), dtype=torch.float64, device=system.device)
    A.check(lib.gmnn_last_layer_features(C.byref(mc), C.byref(sc), C.byref(nc), flags, _ptr(phi), _ptr(ws), nbytes,
                                         _stream()), "gmnn_last_layer_features")
    return phi


def select_max_distance(pool: torch.Tensor, n_select: int, train: torch.Tensor | None = None) -> torch.Tensor:
    """Greedy maximum-distance selection of n_select rows of pool [n, d]
    (float64 device tensor), against the training rows `train` [t, d]; the
    picked row indices in order (int32 device tensor)."""
    pool = pool.to(torch.float64).contiguous()
    n, d = pool.shape
    tr = None if train is None else train.to(device=pool.device, dtype=torch.float64).contiguous()
    lib = A.load()
    nbytes = lib.gmnn_select_workspace_bytes(n)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=pool.device)
    out = torch.empty(max(n_select, 1), dtype=torch.int32, device=pool.device)
    A.check(lib.gmnn_select_max_distance(_ptr(pool), n, d, None if tr is None else _ptr(tr),
                                         0 if tr is None else tr.shape[0], n_select, _ptr(out), _ptr(ws), nbytes,
                                         _stream()), "gmnn_select_max_distance")
    return out[:n_select]


# ---------------------------------------------------------------------------
# shallow-ensemble training step (gmnn_ensemble_loss, gmnn_backward per head,
# gmnn_adam_step, gmnn_lr_factor)
_LOSS_KIND = {"mse": A.GMNN_LOSS_MSE, "nll": A.GMNN_LOSS_NLL, "crps": A.GMNN_LOSS_CRPS}
GROUPS = ("embedding", "nn", "scale", "shift")


@dataclass
class LossSpec:
    """Energy and force loss terms over the heads: kinds "mse", "nll" or
    "crps", weights, the energy term per atom or not, and the variance floor."""
    energy: str = "crps"
    force: str = "crps"
    w_energy: float = 1.0
    w_force: float = 1.0
    energy_per_atom: bool = True
    var_floor: float = 0.0

    def c(self):
        return A.gmnn_loss(_LOSS_KIND[self.energy], _LOSS_KIND[self.force], int(self.energy_per_atom), 0,
                           float(self.w_energy), float(self.w_force), float(self.var_floor))


def ensemble_loss(system: System, energy, forces_heads, energy_ref, forces_ref, spec: LossSpec, workspace=None):
    """(loss [2] float64 = energy term, force term; dL/dE^m [B, heads] float64;
    dL/dF^m [heads, N, 3] float32), all device tensors, from the per-head
    energies and forces of an evaluation with force_var=True."""
    lib = A.load()
    dev = system.device
    B, N = system.n_structs, system.n_atoms
    energy = energy.to(torch.float64).contiguous()
    M = energy.shape[1]
    fh = forces_heads.to(torch.float32).contiguous()
    if fh.shape[0] != M or fh.shape[1] < N:
        raise ValueError("forces_heads must be [heads, N, 3]")
    if fh.shape[1] != N:
        fh = fh[:, :N].contiguous()
    er = torch.as_tensor(energy_ref, dtype=torch.float64, device=dev).contiguous()
    fr = torch.as_tensor(forces_ref, dtype=torch.float32, device=dev).reshape(-1, 3)[:N].contiguous()
    sc = system.c()
    nbytes = lib.gmnn_loss_workspace_bytes(C.byref(sc))
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    loss = torch.empty(2, dtype=torch.float64, device=dev)
    dE = torch.empty((B, M), dtype=torch.float64, device=dev)
    dF = torch.empty((M, max(N, 1), 3), dtype=torch.float32, device=dev)
    lc = spec.c()
    A.check(lib.gmnn_ensemble_loss(C.byref(lc), C.byref(sc), M, _ptr(energy), _ptr(fh), _ptr(er), _ptr(fr),
                                   _ptr(loss), _ptr(dE), _ptr(dF), _ptr(workspace), nbytes, _stream()),
            "gmnn_ensemble_loss")
    return loss, dE, dF


def lr_factor(kind: str = "constant", step: int = 0, total_steps: int = 1, end_factor: float = 0.0,
              period: int = 1, decay_factor: float = 1.0) -> float:
    """Learning-rate multiplier of a schedule at a 0-based step (gmnn_lr_factor)."""
    k = {"constant": A.GMNN_LR_CONSTANT, "linear": A.GMNN_LR_LINEAR, "cosine": A.GMNN_LR_COSINE}[kind]
    sc = A.gmnn_lr_schedule(k, 0, int(total_steps), float(end_factor), int(period), float(decay_factor))
    return float(A.load().gmnn_lr_factor(C.byref(sc), int(step)))


class Adam:
    """On-device Adam (gmnn_adam_step) over a Model's parameters, one learning
    rate per group ("embedding", "nn", "scale", "shift"), optionally scaled
    by a schedule (a dict of lr_factor's keyword arguments).  Updates the
    model's tensors in place and re-packs its weights."""

    def __init__(self, model: Model, lr: dict, betas=(0.9, 0.999), eps: float = 1e-8, schedule: dict | None = None):
        self.model = model
        self.lr = {g: float(lr.get(g, 0.0)) for g in GROUPS}
        self.betas, self.eps, self.schedule = betas, eps, schedule
        self.t = 0
        self.m1 = {k: torch.zeros_like(v) for k, v in model.tensors.items()}
        self.m2 = {k: torch.zeros_like(v) for k, v in model.tensors.items()}
        self._c1 = A.gmnn_param_grads(*[_ptr(self.m1[k]) for k in PARAM_NAMES])
        self._c2 = A.gmnn_param_grads(*[_ptr(self.m2[k]) for k in PARAM_NAMES])

    def step(self, grads: dict):
        f = 1.0 if self.schedule is None else lr_factor(step=self.t, **self.schedule)
        self.t += 1
        opt = A.gmnn_adam((C.c_double * 4)(*[self.lr[g] * f for g in GROUPS]), self.betas[0], self.betas[1],
                          self.eps, self.t)
        gc = A.gmnn_param_grads(*[_ptr(grads[k]) for k in PARAM_NAMES])
        self.model.ensure_packed()
        mc = self.model.c()
        A.check(A.load().gmnn_adam_step(C.byref(mc), C.byref(gc), C.byref(self._c1), C.byref(self._c2),
                                        C.byref(opt), _stream()), "gmnn_adam_step")


class EnsembleTrainer:
    """One on-device training step of a shallow ensemble (Section 2.2 losses,
    Section 3.4 optimiser): per-head energies and forces (force_var
    evaluation), the loss terms and their per-head gradients, the per-head
    double backward, the Adam update.  No host synchronisation; step()
    returns the device loss terms of the evaluated (pre-update) parameters."""

    def __init__(self, model: Model, system: System, nl: NeighborList, energy_ref, forces_ref, loss: LossSpec,
                 adam: Adam, precision: str = "fp32", plan=None):
        self.model, self.system, self.nl, self.loss, self.adam = model, system, nl, loss, adam
        self.precision = precision
        dev = system.device
        self.energy_ref = torch.as_tensor(energy_ref, dtype=torch.float64, device=dev).contiguous()
        self.forces_ref = torch.as_tensor(forces_ref, dtype=torch.float32, device=dev).reshape(-1, 3).contiguous()
        self.ev = EnergyForces(model, system, nl, precision=precision, stress=False, force_var=True, plan=plan)
        self.grads = {k: torch.empty_like(v) for k, v in model.tensors.items()}
        lib = A.load()
        mc, sc, nc = model.c(), system.c(), nl.c()
        flags = A.GMNN_BACKWARD_PER_HEAD | (A.GMNN_PREC_BF16 if precision == "bf16" else 0)
        nb = lib.gmnn_workspace_bytes(A.GMNN_OP_BACKWARD, C.byref(mc), C.byref(sc), C.byref(nc), flags)
        self._bws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        self._lws = torch.empty(max(lib.gmnn_loss_workspace_bytes(C.byref(sc)), 1), dtype=torch.uint8, device=dev)

    def step(self):
        out = self.ev()
        loss, dE, dF = ensemble_loss(self.system, out.energy, out.forces_heads, self.energy_ref, self.forces_ref,
                                     self.loss, workspace=self._lws)
        param_grads(self.model, self.system, self.nl, dE, dF, workspace=self._bws, precision=self.precision,
                    out=self.grads, per_head=True)
        self.adam.step(self.grads)
        return loss
