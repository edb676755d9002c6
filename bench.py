"""Throughput of the GMNN energy+force hot path on one MI355X.

A step is one full pass of the path (pair moments -> invariants -> network
forward and backward -> invariant backward -> pair backward -> force gather
-> FP64 per-structure sums) over the workload, with the neighbour list built
once beforehand (it is reused across steps, as in MD between rebuilds) and
all inputs resident in HBM.  The K steps are timed twice: launched one call
at a time, and replayed from HIP graphs of 10 evaluations each (the way a
loop over fixed buffers drives the library); the faster is the step time.
The headline value is the BF16-network path; the plain FP32 path is timed
the same way and reported beside it, each with its error against the FP64
oracle on the same inputs.

The default workload is the 100,000-atom solid-like lattice (2x512 network,
r_c 6 A, list built at r_c + 1 A skin).  Its errors against FP64 come from
sampled atoms: the oracle evaluates non-periodic cluster cuts around a few
atoms, whose inner atoms carry their periodic energies and forces.  Whole MD
steps (velocity Verlet in a HIP graph, list rebuilds included) are timed on
the same box and reported beside the evaluation.

    python bench.py [--steps K] [--warmup W] [--workload solid]

Prints one JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "energy+force atom-evals/s on 1 GPU, fused BF16 vs plain FP32, at force err vs FP64"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}
# the stages gmnn_energy_forces_timed brackets with events (GMNN_TIMED_STAGES)
STAGES = ["pair_moments", "readout_features", "readout_network", "readout_backward", "pair_backward", "finish"]
GRAPH_EVALS = 10  # evaluations per HIP graph in the graph-launched timing


class HipEvents:
    """hipEvent_t handles through the HIP runtime (recorded by the library on
    the stream its kernels run on)."""

    def __init__(self):
        self.rt = C.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.rt.hipEventDestroy.argtypes = [C.c_void_p]
        self.rt.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]

    def create(self, n):
        arr = (C.c_void_p * n)()
        for k in range(n):
            h = C.c_void_p()
            assert self.rt.hipEventCreate(C.byref(h)) == 0
            arr[k] = h
        return arr

    def record(self, ev, stream):
        assert self.rt.hipEventRecord(ev, stream) == 0

    def elapsed_ms(self, a, b):
        ms = C.c_float()
        assert self.rt.hipEventElapsedTime(C.byref(ms), a, b) == 0
        return ms.value

    def destroy(self, arr):
        for h in arr:
            self.rt.hipEventDestroy(h)


def algorithmic_work(spec, n_atoms, n_pairs):
    """Bytes (HBM-bound stages) or flops (network) one launch must move/do."""
    H1, H2 = spec.hidden
    F, M = spec.n_features, spec.n_heads
    mlp_flops = 2 * (F * H1 + H1 * H2 + H2 * M) + 2 * (H2 * H1 + H1 * F)
    return {
        # j + packed shift per pair; per atom: pos, species, row_ptr, structure id, moments out
        "pair_moments": ("hbm", 8 * n_pairs + n_atoms * (12 + 4 + 8 + 4 + 400)),
        # the network (forward and input gradient) dominates the readout kernels
        "readout_tile": ("mfma", mlp_flops * n_atoms),
        "readout_network": ("mfma", mlp_flops * n_atoms),
        # moments in (400 B), invariants out (1536 B: FP32, or bf16 high + low parts)
        "readout_features": ("hbm", n_atoms * (400 + 1536)),
        # moments and dE/dG in, dE/dPsi out
        "readout_backward": ("hbm", n_atoms * (400 + 4 * 384 + 400)),
        # list + g out per pair; per atom: moment gradient in, virial out, pos, species, row_ptr
        "pair_backward": ("hbm", 20 * n_pairs + n_atoms * (400 + 36 + 12 + 4 + 8 + 4)),
        # the fused tile kernel does moments + readout + pair backward; its
        # dense work is the network on MFMA
        "fused_tile": ("mfma", mlp_flops * n_atoms),
        # rev + two g reads per pair; forces out; per-structure sums read E_i and virials
        "finish": ("hbm", 28 * n_pairs + n_atoms * (12 + 8 + 4 * M + 36)),
    }


def kernel_source_hash():
    """SHA-256 over the HIP sources (and the C header) that make up libgmnn.so."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_22168_amd", "csrc")
    files = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".h")))
    for f in files + ["../../include/gmnn.h"]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def plan_tag(plan):
    """Short name of an execution plan: fused8 / fused16 / split-tile / split-stream."""
    if plan["schedule"] == 1:
        return f"fused{plan['tile_atoms']}"
    return "split-stream" if plan["readout"] == 2 else "split-tile"


def counted_traffic(workload, stage, precision, plan):
    """HBM bytes per launch of a stage as counted by rocprofv3 (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy) from the summary committed under
    profiles/, or None when that summary was taken on other kernel sources
    or under another execution plan."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_counters.md")
    try:
        text = open(path).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        data = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if data.get("source_sha256") != kernel_source_hash():
        return None
    entry = data.get("stages", {}).get(f"{workload}:{stage}:{precision}:{plan_tag(plan)}")
    return None if entry is None else entry["fetch_bytes"] + entry["write_bytes"]


def run_path(g, A, model, system, nl, precision, steps, warmup, events, plan="auto", force_var=False):
    import torch
    ev = g.EnergyForces(model, system, nl, precision=precision, stress=True, force_var=force_var, plan=plan)
    for _ in range(warmup):
        ev()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ev()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-stage durations: the same steps again with events around each kernel
    lib = A.load()
    evs = [events.create(2 * len(STAGES)) for _ in range(steps)]
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for k in range(steps):
        st = lib.gmnn_energy_forces_timed(C.byref(ev._mc), C.byref(ev._sc), C.byref(ev._nc), ev.flags,
                                          None if ev._plan is None else C.byref(ev._plan), C.byref(ev._oc),
                                          C.c_void_p(ev.workspace.data_ptr()), ev.ws_bytes, stream, evs[k])
        A.check(st, "gmnn_energy_forces_timed")
    torch.cuda.synchronize()
    stage_ms = {name: float(np.mean([events.elapsed_ms(e[2 * s], e[2 * s + 1]) for e in evs]))
                for s, name in enumerate(STAGES)}

    # cost of an event bracket around nothing (the same stream, same steps)
    empty = []
    for _ in range(steps):
        e = events.create(2)
        events.record(e[0], stream)
        events.record(e[1], stream)
        empty.append(e)
    torch.cuda.synchronize()
    overhead = float(np.median([events.elapsed_ms(e[0], e[1]) for e in empty]))
    for e in empty:
        events.destroy(e)
    if ev.plan["schedule"] == A.GMNN_SCHEDULE_FUSED:
        # small systems run moments, readout and pair backward in one launch
        stage_ms = {"fused_tile": stage_ms["pair_moments"], "finish": stage_ms["finish"]}
    elif ev.plan["readout"] != A.GMNN_READOUT_STREAM:
        # the tile readout is one kernel (invariants, network, invariant backward)
        stage_ms = {"pair_moments": stage_ms["pair_moments"], "readout_tile": stage_ms["readout_features"],
                    "pair_backward": stage_ms["pair_backward"], "finish": stage_ms["finish"]}
    stage_ms = {k: max(v - overhead, 0.0) for k, v in stage_ms.items()}
    stage_ms["_event_overhead"] = overhead
    # each step on its own between two events (nothing else inside): median and
    # interquartile range, the empty-bracket cost subtracted
    brackets = [events.create(2) for _ in range(steps)]
    torch.cuda.synchronize()
    for e in brackets:
        events.record(e[0], stream)
        ev()
        events.record(e[1], stream)
    torch.cuda.synchronize()
    per_step = np.array([events.elapsed_ms(e[0], e[1]) for e in brackets]) - overhead
    for e in brackets:
        events.destroy(e)
    q1, med, q3 = np.percentile(per_step, [25, 50, 75])
    for e in evs:
        events.destroy(e)
    out = ev(sync=True)
    stage_ms["_plan"] = ev.plan
    stage_ms["_step_stats"] = {"median_us": med * 1e3, "iqr_us": (q3 - q1) * 1e3, "n": int(len(per_step))}
    # the same K steps replayed from HIP graphs of GRAPH_EVALS evaluations each
    per = GRAPH_EVALS if steps % GRAPH_EVALS == 0 else 1
    ev.capture(per)
    ev.replay(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev.replay(steps // per)
    torch.cuda.synchronize()
    stage_ms["_graph_wall"] = time.perf_counter() - t0
    ev.release()
    return wall, stage_ms, out


def errors_vs_oracle(out, ref, n_atoms, nb):
    F = out.forces.cpu().numpy()[:n_atoms].astype(np.float64)
    dF = F - ref.forces
    E = out.energy.cpu().numpy()
    rmsF = float(np.sqrt((ref.forces ** 2).mean()))
    return {
        "force_mae": float(np.abs(dF).mean()), "force_rmse": float(np.sqrt((dF ** 2).mean())),
        "force_max": float(np.abs(dF).max()), "force_rmse_rel": float(np.sqrt((dF ** 2).mean()) / rmsF),
        "energy_per_atom_max": float((np.abs(E - ref.energy) / nb[:, None]).max()),
        "stress_max": float(np.abs(out.stress.cpu().numpy() - ref.stress).max()),
        "rms_force": rmsF,
    }


def sampled_errors(outs, batch, params, spec, centers, margin=3.0):
    """Errors against the FP64 oracle on sampled atoms of a structure too
    large to evaluate whole: the oracle evaluates a non-periodic cluster of
    radius 2 r_c + margin around each centre; the cluster atoms within
    `margin` of the centre carry their periodic forces, those within
    r_c + margin their periodic energies."""
    from oracle import brute_force_neighbors, evaluate
    from workloads import cluster_cut
    rc = spec.model.r_cut
    R = 2.0 * rc + margin
    refs = []
    for c in centers:
        cut, idx, dist = cluster_cut(batch, int(c), R)
        refs.append((idx, dist, evaluate(cut, params, brute_force_neighbors(cut, rc), want_stress=False)))
    res = {}
    N = batch.n_atoms
    for prec, o in outs.items():
        F = o.forces.cpu().numpy()[:N].astype(np.float64)
        Ei = o.atomic_energy.cpu().numpy()[:N].astype(np.float64)
        dF, Fr, dE = [], [], []
        for idx, dist, r in refs:
            fi, ei = dist < R - 2 * rc, dist < R - rc
            dF.append(F[idx[fi]] - r.forces[fi])
            Fr.append(r.forces[fi])
            dE.append(Ei[idx[ei]] - r.atomic[ei])
        dF, Fr, dE = np.concatenate(dF), np.concatenate(Fr), np.concatenate(dE)
        rms = float(np.sqrt((Fr ** 2).mean()))
        res[prec] = {"force_mae": float(np.abs(dF).mean()), "force_rmse": float(np.sqrt((dF ** 2).mean())),
                     "force_max": float(np.abs(dF).max()), "force_rmse_rel": float(np.sqrt((dF ** 2).mean()) / rms),
                     "atomic_energy_max": float(np.abs(dE).max()), "rms_force": rms,
                     "sampled": f"forces of {len(dF)} atoms and energies of {len(dE)} atoms: the inner atoms of "
                                f"{len(centers)} cluster cuts of radius {R:.1f} A evaluated by the FP64 oracle"}
    return res


def time_neighbor_build(g, A, system, nl, cutoff, skin, events, reps=20):
    """The neighbour list build on its own (reported beside the evaluation):
    median and IQR of hipEvent-timed rebuilds into the same list."""
    import torch
    lib = A.load()
    sysc = system.c()
    nbytes = lib.gmnn_neighbors_workspace_bytes(C.byref(sysc), cutoff, skin)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=system.device)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ts = []
    for k in range(reps + 3):
        e = events.create(2)
        events.record(e[0], stream)
        nlc = nl.c()
        A.check(lib.gmnn_build_neighbors(C.byref(sysc), cutoff, skin, C.byref(nlc), 0, C.c_void_p(ws.data_ptr()),
                                         nbytes, stream), "gmnn_build_neighbors")
        events.record(e[1], stream)
        torch.cuda.synchronize()
        if k >= 3:
            ts.append(events.elapsed_ms(e[0], e[1]))
        events.destroy(e)
    q1, med, q3 = np.percentile(ts, [25, 50, 75])
    return {"median_us": med * 1e3, "iqr_us": (q3 - q1) * 1e3, "reps": reps, "cutoff_plus_skin": cutoff + skin,
            "n_pairs": nl.n_pairs}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, params, nl_ref, budget_s, what=None):
    """The FP64 oracle (energy, forces, stress; list excluded) on the host
    cores, repeated for about budget_s seconds with all threads, then for half
    that with one thread (reported beside it)."""
    import torch
    from oracle import evaluate

    def run(budget):
        reps = 0
        t0 = time.perf_counter()
        while True:
            evaluate(batch, params, nl_ref)
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return reps, el
    cores = torch.get_num_threads()
    reps, el = run(budget_s)
    torch.set_num_threads(1)
    try:
        reps1, el1 = run(budget_s / 2)
    finally:
        torch.set_num_threads(cores)
    return {"value": batch.n_atoms * reps / el, "unit": "atom-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} FP64 oracle evaluations (energy, forces, stress; list excluded) of "
                      f"{what or f'the {batch.n_atoms}-atom workload'}, {el:.1f} s",
            "cpu_model": _cpu_model(), "value_1_thread": batch.n_atoms * reps1 / el1}


def measure_md(workload, steps, graph_steps, sigma0, precisions=("bf16", "fp32")):
    """NVE velocity-Verlet MD of the workload (skin list, HIP graph of
    graph_steps steps replayed); atom-steps/s of whole MD steps including
    list rebuilds, as MD step time is quoted per atom and step."""
    import torch
    import paper_2505_22168_amd as g
    from workloads import make_workload
    import dataclasses
    from workloads.configs import make_params
    masses_by_species = {0: 6.94, 1: 30.974, 2: 15.999, 3: 12.011, 4: 1.008}
    batch, params, spec = make_workload(workload)
    # random weights make an unphysical potential: the species scale sigma0
    # sets the force magnitude (the arithmetic per step does not depend on it)
    params = make_params(dataclasses.replace(spec.model, sigma0=sigma0), spec.seed + 1000)
    masses = np.array([masses_by_species[int(z) % 5] for z in batch.species])
    v0 = g.maxwell_boltzmann(masses, 600.0, seed=3)
    system = g.System.from_batch(batch, "cuda")
    model = g.Model.from_params(params, "cuda")
    skin = spec.skin if spec.skin > 0 else 1.0
    out = {}
    for prec in precisions:
        system.pos.copy_(torch.as_tensor(batch.pos, device="cuda"))
        md = g.MD(model, system, masses, dt=0.5, skin=skin, velocities=v0, precision=prec)
        e0 = float(md.energy.sum().item()) + md.kinetic_energy(masses)
        gs = graph_steps
        md.capture(gs)
        md.run(1)  # warm-up replay
        torch.cuda.synchronize()
        reps = max(1, steps // gs)
        t0 = time.perf_counter()
        md.run(reps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ke1 = md.kinetic_energy(masses)
        e1 = float(md.energy.sum().item()) + ke1
        t1 = 2.0 * ke1 / (3.0 * batch.n_atoms * g.api.KB_EV_PER_K)
        nsteps = reps * gs
        out[prec] = {"value": batch.n_atoms * nsteps / wall, "ms_per_step": wall / nsteps * 1e3,
                     "us_per_atom_step": wall / nsteps / batch.n_atoms * 1e6, "steps": nsteps + gs,
                     "status": md.status(), "total_energy_drift_eV_per_atom": (e1 - e0) / batch.n_atoms,
                     "finite": bool(torch.isfinite(system.pos).all().item()), "T_final_K": t1}
        print(f"[bench-md] {prec}: {out[prec]}", file=sys.stderr, flush=True)
        md.release()
    return out, batch, spec, skin


def run_md(args):
    out, batch, spec, skin = measure_md(args.workload, args.steps, args.graph_steps, args.md_sigma0)
    line = {"metric": "MD atom-steps/s (NVE velocity Verlet, HIP graph, skin list)", "value": out["bf16"]["value"],
            "unit": "atom-steps/s", "n_gpus": 1, "steps": out["bf16"]["steps"], "dtype": "bf16",
            "config": {"workload": args.workload, "n_atoms": batch.n_atoms, "dt_fs": 0.5, "skin": skin,
                       "graph_steps": args.graph_steps, "mlp": list(spec.model.hidden), "sigma0": args.md_sigma0,
                       "T0_K": 600.0},
            "bf16": out["bf16"], "fp32": out["fp32"]}
    print(json.dumps(line))


def _wall(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def run_ensemble(args):
    """Shallow-ensemble batched inference: all structures of the workload in
    one launch sequence (head-mean energy and forces, energy variance, per-atom
    force variance from one backward per head) vs the same evaluation issued
    structure by structure."""
    import torch
    import paper_2505_22168_amd as g
    from workloads import make_workload
    name = args.workload if args.workload not in ("liquid", "solid") else "ensemble"
    batch, params, spec = make_workload(name)
    dev = torch.device("cuda:0")
    model = g.Model.from_params(params, dev)
    system = g.System.from_batch(batch, dev)
    nl = g.build_neighbors(system, spec.model.r_cut, spec.skin)
    plan = None if args.plan == "builtin" else "auto"
    out = {}
    for prec in ("bf16", "fp32"):
        ev = g.EnergyForces(model, system, nl, precision=prec, stress=True, force_var=True, plan=plan)
        t_batched = _wall(ev, args.steps, args.warmup)
        per = []
        for b in range(batch.n_structs):
            sb = batch.structure(b)
            s_sys = g.System.from_batch(sb, dev)
            s_nl = g.build_neighbors(s_sys, spec.model.r_cut, spec.skin)
            per.append(g.EnergyForces(model, s_sys, s_nl, precision=prec, stress=True, force_var=True, plan=plan))

        def all_structs():
            for e in per:
                e()
        t_per = _wall(all_structs, max(1, args.steps // 5), 2)
        # the two must agree (same kernels, same order within a structure)
        o = ev(sync=True)
        e_b = o.energy.cpu().numpy()
        e_s = np.concatenate([e(sync=True).energy.cpu().numpy() for e in per])
        out[prec] = {"batched_ms": t_batched * 1e3, "per_structure_ms": t_per * 1e3,
                     "batched_atom_evals_per_s": batch.n_atoms / t_batched,
                     "per_structure_atom_evals_per_s": batch.n_atoms / t_per, "speedup": t_per / t_batched,
                     "plan": ev.plan, "energy_max_abs_diff_batched_vs_single": float(np.abs(e_b - e_s).max())}
        print(f"[bench-ensemble] {prec}: {out[prec]}", file=sys.stderr, flush=True)
    line = {"metric": "shallow-ensemble energy+force(+variance) atom-evals/s, batched vs per-structure",
            "value": out["bf16"]["batched_atom_evals_per_s"], "unit": "atom-evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": name, "n_atoms": batch.n_atoms, "n_structs": batch.n_structs,
                       "n_pairs": nl.n_pairs, "heads": spec.model.n_heads, "mlp": list(spec.model.hidden)},
            "bf16": out["bf16"], "fp32": out["fp32"]}
    print(json.dumps(line))


def run_train(args):
    """Training-gradient step of the energy+force loss: energies and forces,
    then the loss gradients w.r.t. every parameter (double backward), with the
    network products in BF16 (headline) and in FP32."""
    import torch
    import paper_2505_22168_amd as g
    from workloads import make_workload
    name = args.workload if args.workload not in ("liquid", "solid") else "train"
    batch, params, spec = make_workload(name)
    dev = torch.device("cuda:0")
    model = g.Model.from_params(params, dev)
    system = g.System.from_batch(batch, dev)
    nl = g.build_neighbors(system, spec.model.r_cut, spec.skin)
    rng = np.random.default_rng(7)
    dE = torch.as_tensor(rng.normal(size=batch.n_structs), device=dev)
    dF = torch.as_tensor(rng.normal(size=(batch.n_atoms, 3)).astype(np.float32), device=dev)
    lib = g.load_library()
    from paper_2505_22168_amd import _capi as A
    nbytes = lib.gmnn_workspace_bytes(A.GMNN_OP_BACKWARD, C.byref(model.c()), C.byref(system.c()),
                                      C.byref(nl.c()), 0)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    res = {}
    grads = {}
    for prec in ("bf16", "fp32"):
        ev = g.EnergyForces(model, system, nl, precision=prec, stress=False)
        gout = {k: torch.empty_like(v) for k, v in model.tensors.items()}

        def step():
            ev()
            return g.param_grads(model, system, nl, dE, dF, workspace=ws, precision=prec, out=gout)
        t = _wall(step, args.steps, args.warmup)
        t_fwd = _wall(ev, args.steps, args.warmup)
        grads[prec] = step()
        res[prec] = {"value": batch.n_atoms / t, "ms_per_step": t * 1e3, "forward_ms": t_fwd * 1e3,
                     "backward_ms": (t - t_fwd) * 1e3}
        print(f"[bench-train] {prec}: {res[prec]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # BF16 gradients against the FP32 path's (relative l2 per parameter)
    diff = {k: float(torch.linalg.norm((grads["bf16"][k] - grads["fp32"][k]).double())
                     / max(float(torch.linalg.norm(grads["fp32"][k].double())), 1e-30)) for k in grads["fp32"]}
    line = {"metric": "training-gradient atom-evals/s (energy+forces, then parameter gradients of an "
                      "energy+force loss)", "value": res["bf16"]["value"], "unit": "atom-evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["bf16"]["ms_per_step"], "dtype": "bf16",
            "data": "synthetic", "bf16": res["bf16"], "fp32": res["fp32"], "bf16_grad_rel_diff_vs_fp32": diff,
            "config": {"workload": name, "n_atoms": batch.n_atoms, "n_structs": batch.n_structs,
                       "n_pairs": nl.n_pairs, "mlp": list(spec.model.hidden)}}
    print(json.dumps(line))


def run_train_ensemble(args):
    """One whole on-device training step of a shallow ensemble (Section 2.2,
    Section 3.4): per-head energies and forces, CRPS loss terms on energies
    per atom and force components, the per-head double backward, one Adam
    update with four parameter groups.  Training batch of 32 structures of
    U{100..600} atoms with the 16-head 2x256 shallow-ensemble network."""
    import dataclasses
    import torch
    import paper_2505_22168_amd as g
    from workloads import make_workload, make_params
    batch, _, spec = make_workload("train")
    ens = make_workload("ensemble", n_structs=1)[2]
    mspec = dataclasses.replace(spec.model, hidden=ens.model.hidden, n_heads=ens.model.n_heads)
    params = make_params(mspec, 31)
    dev = torch.device("cuda:0")
    system = g.System.from_batch(batch, dev)
    nl = g.build_neighbors(system, mspec.r_cut, spec.skin)
    rng = np.random.default_rng(7)
    nb = np.diff(batch.atom_ptr)
    Er = -3.0 * nb + rng.normal(size=batch.n_structs) * np.sqrt(nb) * 0.05
    Fr = rng.normal(size=(batch.n_atoms, 3)).astype(np.float32)
    res = {}
    for prec in ("bf16", "fp32"):
        model = g.Model(mspec, params.as_dict(), dev)
        adam = g.Adam(model, {"embedding": 5e-4, "nn": 5e-4, "scale": 5e-4, "shift": 5e-4},
                      schedule=dict(kind="linear", total_steps=1000, end_factor=0.1))
        tr = g.EnsembleTrainer(model, system, nl, Er, Fr, g.LossSpec("crps", "crps", 1.0, 1.0, True, 1e-6), adam,
                               precision=prec)
        t = _wall(tr.step, args.steps, args.warmup)
        t_fwd = _wall(tr.ev, args.steps, args.warmup)
        out = tr.ev()
        t_loss = _wall(lambda: g.ensemble_loss(system, out.energy, out.forces_heads, tr.energy_ref, tr.forces_ref,
                                               tr.loss, workspace=tr._lws), args.steps, args.warmup)
        loss, dE, dF = g.ensemble_loss(system, out.energy, out.forces_heads, tr.energy_ref, tr.forces_ref, tr.loss)
        t_bwd = _wall(lambda: g.param_grads(model, system, nl, dE, dF, workspace=tr._bws, precision=prec,
                                            out=tr.grads, per_head=True), args.steps, args.warmup)
        t_adam = _wall(lambda: adam.step(tr.grads), args.steps, args.warmup)
        l0 = tr.step().cpu().numpy()
        res[prec] = {"value": batch.n_atoms / t, "ms_per_step": t * 1e3, "forward_ms": t_fwd * 1e3,
                     "loss_ms": t_loss * 1e3, "backward_ms": t_bwd * 1e3, "adam_ms": t_adam * 1e3,
                     "loss_terms_after_timing": [float(l0[0]), float(l0[1])]}
        print(f"[bench-train-ensemble] {prec}: {res[prec]}", file=sys.stderr, flush=True)
    line = {"metric": "shallow-ensemble training-step atom-evals/s (per-head forces, CRPS loss, per-head double "
                      "backward, Adam)", "value": res["bf16"]["value"], "unit": "atom-evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["bf16"]["ms_per_step"], "dtype": "bf16",
            "data": "synthetic", "bf16": res["bf16"], "fp32": res["fp32"],
            "config": {"workload": "train batch, 16-head ensemble network", "n_atoms": batch.n_atoms,
                       "n_structs": batch.n_structs, "n_pairs": nl.n_pairs, "mlp": list(mspec.hidden),
                       "heads": mspec.n_heads}}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="solid")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--md-steps", type=int, default=200,
                    help="whole MD steps timed beside the evaluation (0: none)")
    ap.add_argument("--no-oracle", action="store_true", help="skip oracle errors and the CPU baseline")
    ap.add_argument("--md", action="store_true", help="time whole MD steps instead (not the headline metric)")
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--md-sigma0", type=float, default=0.003, help="species energy scale of the MD model")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (reference for HBM byte counters)")
    ap.add_argument("--plan", default="auto", choices=["auto", "builtin"],
                    help="execution plan: autotuned (cached per shape class) or the library's built-in choice")
    ap.add_argument("--ensemble", action="store_true",
                    help="C5 mode: one batched launch (heads, energy/force variance) vs per-structure launches")
    ap.add_argument("--train", action="store_true",
                    help="training-gradient mode: energy+forces then gmnn_backward per step (FP32)")
    ap.add_argument("--train-ensemble", action="store_true",
                    help="whole shallow-ensemble training steps (per-head forces, CRPS loss, backward, Adam)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library runs on one GPU (no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": args.steps}))
        return
    if args.md:
        return run_md(args)
    if args.plan == "auto" and "GMNN_TUNE_CACHE" not in os.environ:
        import tempfile
        os.environ["GMNN_TUNE_CACHE"] = os.path.join(tempfile.gettempdir(), f"gmnn_tune_{os.getpid()}.json")
    if args.ensemble:
        return run_ensemble(args)
    if args.train:
        return run_train(args)
    if args.train_ensemble:
        return run_train_ensemble(args)
    import torch
    import paper_2505_22168_amd as g
    from paper_2505_22168_amd import _capi as A
    from workloads import make_workload

    g.load_library()
    batch, params, spec = make_workload(args.workload)
    dev = torch.device("cuda:0")
    system = g.System.from_batch(batch, dev)
    nl = g.build_neighbors(system, spec.model.r_cut, spec.skin)
    model = g.Model.from_params(params, dev)
    events = HipEvents()
    nl_stats = time_neighbor_build(g, A, system, nl, spec.model.r_cut, spec.skin, events)
    N, P = batch.n_atoms, nl.n_pairs
    print(f"[bench] workload {args.workload}: {N} atoms, {P} pairs, {batch.n_structs} structures", file=sys.stderr,
          flush=True)

    res = {}
    eager_ms, graph_ms, step_stats = {}, {}, {}
    for prec in ("bf16", "fp32"):
        wall, stage_ms, out = run_path(g, A, model, system, nl, prec, args.steps, args.warmup, events,
                                       plan=None if args.plan == "builtin" else "auto")
        plan = stage_ms.pop("_plan")
        gwall = stage_ms.pop("_graph_wall")
        step_stats[prec] = stage_ms.pop("_step_stats")
        res[prec] = (min(wall, gwall), stage_ms, out, plan)
        eager_ms[prec] = wall / args.steps * 1e3
        graph_ms[prec] = gwall / args.steps * 1e3
        print(f"[bench] {prec}: {wall / args.steps * 1e3:.4f} ms/step eager, {gwall / args.steps * 1e3:.4f} ms/step "
              f"graph-launched, plan {plan}, stages(us) "
              + ", ".join(f"{k}={v * 1e3:.1f}" for k, v in stage_ms.items()), file=sys.stderr, flush=True)

    wall, stage_ms, out16, plan16 = res["bf16"]
    ms_per_step = wall / args.steps * 1e3
    value = N * args.steps / wall
    work = algorithmic_work(spec.model, N, P)
    overhead_ms = stage_ms.pop("_event_overhead")
    res["fp32"][1].pop("_event_overhead", None)
    dom = max(stage_ms, key=stage_ms.get)
    bound, amount = work[dom]
    dur_s = stage_ms[dom] * 1e-3
    if bound == "hbm":
        achieved, peak, unit = amount / dur_s / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = amount / dur_s / 1e12, MFMA_PEAK_TFLOPS["bf16"], "TFLOP/s"
    roofline = {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": counted_traffic(args.workload, dom, "bf16", plan16),
                "per_launch": {"amount": amount, "what": "bytes" if bound == "hbm" else "flops",
                               "avg_duration_us": stage_ms[dom] * 1e3,
                               "event_bracket_overhead_us_subtracted": overhead_ms * 1e3}}

    # every stage against its own bound (algorithmic work / event-timed duration)
    stage_roofline = {}
    for k, ms in stage_ms.items():
        b, amt = work[k]
        if ms > 0:
            stage_roofline[k] = {"bound": b, "frac": (amt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if b == "hbm"
                                 else (amt / (ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["bf16"])}

    wall32, stage32, out32, plan32 = res["fp32"]
    fp32 = {"value": N * args.steps / wall32, "ms_per_step": wall32 / args.steps * 1e3,
            "stages_us": {k: v * 1e3 for k, v in stage32.items()}, "plan": plan32,
            "ms_per_step_eager": eager_ms["fp32"], "ms_per_step_graph": graph_ms["fp32"]}

    md = None
    if args.md_steps > 0 and spec.skin > 0:
        md_out, _, _, md_skin = measure_md(args.workload, args.md_steps, min(args.graph_steps, args.md_steps),
                                           args.md_sigma0)
        md = {"what": f"whole NVE velocity-Verlet steps (dt 0.5 fs, skin {md_skin} A, list rebuilds decided on the "
                      f"device) in HIP graphs of {min(args.graph_steps, args.md_steps)} steps; species energy scale "
                      f"{args.md_sigma0} keeps the random-weight potential stable (same arithmetic per step)",
              **md_out}

    accuracy = None
    cpu = None
    if not args.no_oracle:
        from oracle import brute_force_neighbors
        t0 = time.perf_counter()
        outs = {"bf16": out16, "fp32": res["fp32"][2]}
        if N > 20000:
            # too large for one oracle evaluation: sampled atoms (cluster cuts)
            centers = np.random.default_rng(11).choice(N, 3, replace=False)
            accuracy = sampled_errors(outs, batch, params, spec, centers)
            # the CPU baseline: the oracle on a periodic cut of the same lattice
            # (same density, species ratio, cutoff and network)
            cut_kw = {"solid": dict(reps=(10, 10, 8))}.get(args.workload, {})
            cb, cp, cs = make_workload(args.workload, **cut_kw)
            cnl = brute_force_neighbors(cb, cs.model.r_cut)
            cpu = cpu_baseline(cb, cp, cnl, args.cpu_budget,
                               what=f"a {cb.n_atoms}-atom periodic cut of the same workload (same density, species "
                                    f"ratio, cutoff and network)")
        else:
            from oracle import evaluate
            nl_ref = brute_force_neighbors(batch, spec.model.r_cut)
            ref = evaluate(batch, params, nl_ref)
            nb = np.diff(batch.atom_ptr)
            accuracy = {k: errors_vs_oracle(o, ref, N, nb) for k, o in outs.items()}
            cpu = cpu_baseline(batch, params, nl_ref, args.cpu_budget)
        print(f"[bench] oracle legs in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": value, "unit": "atom-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": N, "n_pairs": P, "n_structs": batch.n_structs,
                   "r_cut": spec.model.r_cut, "mlp": list(spec.model.hidden), "heads": spec.model.n_heads,
                   "features": spec.model.n_features, "parallelism": "single GPU", "plan": plan16,
                   "launch": (f"HIP graph of {GRAPH_EVALS} evaluations" if graph_ms["bf16"] < eager_ms["bf16"]
                              else "eager launches")},
        "ms_per_step_eager": eager_ms["bf16"], "ms_per_step_graph": graph_ms["bf16"],
        "step_event_stats": step_stats, "neighbor_build": nl_stats,
        "roofline": roofline,
        "stage_roofline": stage_roofline,
        "cpu_baseline": cpu,
        "stages_us": {k: v * 1e3 for k, v in stage_ms.items()},
        "fp32": fp32,
        "bf16_over_fp32": value / fp32["value"],
        "accuracy_vs_fp64": accuracy,
        "md": md,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
