"""Plan cache for gmnn_autotune.

The tuner itself is native (gmnn_autotune times every supported execution
plan with hipEvents and returns the fastest).  This module keys its answer by
the shape class of the problem and keeps it in a JSON file, so a process tunes
each shape class once: the key holds the device name, the flags, the model
widths, the species count, and the atom count, largest structure and mean
list length rounded to powers of two (plans differ in launch shape, not in
arithmetic, so nearby sizes share a choice).
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import threading

import torch

from . import _capi as A

_LOCK = threading.Lock()


def default_path() -> str:
    return os.environ.get("GMNN_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gmnn", "autotune.json"))


def _pow2(x: float) -> int:
    return 0 if x <= 0 else 1 << int(round(math.log2(x)))


def shape_key(model, system, nl, flags: int) -> str:
    """Cache key of one evaluation shape (reads the device pair count: syncs)."""
    n = system.n_atoms
    sizes = system.atom_ptr_host[1:] - system.atom_ptr_host[:-1]
    biggest = int(sizes.max()) if len(sizes) else 0
    mean_row = nl.n_pairs / max(n, 1)
    dev = torch.cuda.get_device_name(system.device)
    s = model.spec
    return "|".join(str(v) for v in ("plan4", dev, flags & ~A.GMNN_SYNC, s.n_species, s.hidden[0], s.hidden[1], s.n_heads,
                                      _pow2(n), _pow2(biggest), _pow2(mean_row)))


class TuneCache:
    """JSON file of shape key -> {"schedule", "lanes_per_atom", "readout", "tile_atoms", "table"}."""

    def __init__(self, path: str | None = None):
        self.path = path or default_path()
        self._data = None

    def _load(self):
        if self._data is None:
            try:
                with open(self.path) as f:
                    self._data = json.load(f)
            except (OSError, ValueError):
                self._data = {}
        return self._data

    def get(self, key: str):
        return self._load().get(key)

    def put(self, key: str, value: dict):
        with _LOCK:
            data = self._load()
            data[key] = value
            os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
            tmp = self.path + f".tmp{os.getpid()}"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def run_autotune(ev, reps: int = 20):
    """gmnn_autotune for an EnergyForces evaluator: returns (plan, table) with
    plan = {"schedule", "lanes_per_atom", "readout", "tile_atoms"} and
    table = [(plan, median_us, min_us)]."""
    lib = A.load()
    best = A.gmnn_plan()
    cap = 32
    entries = (A.gmnn_tune_entry * cap)()
    n = C.c_int32(0)
    st = lib.gmnn_autotune(C.byref(ev._mc), C.byref(ev._sc), C.byref(ev._nc), ev.flags, C.byref(ev._oc),
                           C.c_void_p(ev.workspace.data_ptr()), ev.ws_bytes,
                           C.c_void_p(torch.cuda.current_stream().cuda_stream), reps, C.byref(best), entries, cap,
                           C.byref(n))
    A.check(st, "gmnn_autotune")
    table = [(e.plan.as_dict(), e.median_us, e.min_us) for e in entries[: min(n.value, cap)]]
    return best.as_dict(), table


def tuned_plan(ev, cache: TuneCache | None = None, reps: int = 20) -> dict:
    """The cached plan for ev's shape class, tuning (once) on a miss."""
    cache = cache or TuneCache()
    key = shape_key(ev.model, ev.system, ev.nl, ev.flags)
    hit = cache.get(key)
    if hit is not None:
        return A.gmnn_plan.of(hit).as_dict()
    plan, table = run_autotune(ev, reps)
    cache.put(key, dict(plan, table=[[p[k] for k in A.gmnn_plan.FIELDS] + [med, mn] for p, med, mn in table]))
    return plan
