"""Batched form: several single-brick solvers (uneven meshes, each with its own
drive scenarios) stepped by persistent launches, plus the tile autotuner.

Thin wrapper over pmdg_batch_* of libpmutdg; the solvers stay the owners of
their state and traces."""
import ctypes
import json
import os
import time

from . import _lib
from ._lib import check, lib
from .solver import Solver, _stream_ptr, from_workload

OPT_GRAPH = 1
OPT_TILE_ROWS = 2
OPT_TILE_ZCHUNK = 3
OPT_GRAPH_CHUNK = 4
OPT_TIMING = 5


class Batch:
    def __init__(self, solvers, device="cuda"):
        self.L = lib()
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = ctypes.c_void_p()
        check(self.L.pmdg_batch_create(len(self.solvers), arr, ctypes.byref(h)))
        self.h = h
        self.device = device
        self.ws = None

    def bind(self, stream=None):
        import torch
        n = ctypes.c_size_t()
        check(self.L.pmdg_batch_workspace_size(self.h, ctypes.byref(n)))
        self.ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        check(self.L.pmdg_batch_bind(self.h, ctypes.c_void_p(ptr), n.value, _stream_ptr(stream)))

    def set_option(self, opt, value):
        check(self.L.pmdg_batch_set_option(self.h, int(opt), int(value)))

    def step(self, n, stream=None):
        check(self.L.pmdg_batch_step(self.h, int(n), _stream_ptr(stream)))

    def close(self):
        if getattr(self, "h", None):
            self.L.pmdg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- autotuner

class TileTuner:
    """Picks the stiffness tile shape (rows per wave, planes per z chunk) of a
    mesh by timing candidate shapes with the library's per-kernel HIP events.

    Results are cached per (precision, order, node counts, scenarios) in
    memory and, if a path is given, in a JSON file."""

    def __init__(self, path=None, candidates=None, steps=6):
        self.path = path
        self.steps = steps
        self.cache = {}
        self.candidates = candidates or [(1, 9), (1, 17), (1, 33), (2, 9), (2, 17), (2, 33), (2, 0), (1, 0)]
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    @staticmethod
    def key(dom, S, precision):
        nn = [dom["N"] * e + 1 for e in dom["ne"]]
        return f"p{precision}-N{dom['N']}-{nn[0]}x{nn[1]}x{nn[2]}-S{S}"

    def tune(self, domains, S=1, precision=32):
        if len(domains) != 1:
            raise ValueError("the tuner handles single-brick meshes")
        k = self.key(domains[0], S, precision)
        if k in self.cache:
            return tuple(self.cache[k]["best"])
        import torch
        nz = domains[0]["N"] * domains[0]["ne"][2] + 1
        times = {}
        for rows, zc in self.candidates:
            if zc > nz:
                continue
            s = Solver(domains, precision=precision, n_scenarios=S, trace_capacity=self.steps + 2)
            s.set_option(OPT_TILE_ROWS, rows)
            s.set_option(OPT_TILE_ZCHUNK, zc)
            s.bind()
            s.set_option(OPT_GRAPH, 0)
            s.step(1)
            s.set_option(OPT_TIMING, 1)
            s.step(self.steps)
            times[(rows, zc)] = float(s.kernel_times()[0])
            s.close()
            del s
            torch.cuda.empty_cache()
        best = min(times, key=times.get)
        self.cache[k] = {"best": list(best), "ms": times[best],
                         "all": {f"{r}/{z}": t for (r, z), t in times.items()}}
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return best


def build_batch(workloads, precision=32, shape_fns=None, tuner=None, n_steps=None, device="cuda"):
    """Creates, tunes and binds one solver per workload (all drive rows of each
    become its scenarios), then a bound Batch over them."""
    solvers = []
    for i, wl in enumerate(workloads):
        S = len(wl["drive"]["amp"])
        s = from_workload(wl, precision=precision, n_steps=n_steps, shape_fn=shape_fns[i], device=device,
                          bind=False)
        if tuner is not None:
            rows, zc = tuner.tune(wl["domains"], S=S, precision=precision)
            s.set_option(OPT_TILE_ROWS, rows)
            s.set_option(OPT_TILE_ZCHUNK, zc)
        s.bind()
        solvers.append(s)
    b = Batch(solvers, device=device)
    b.bind()
    return b
