"""Benchmark of the explicit coupled PMUT / DG-SEM step on one MI355X.

Workload: the large-array configuration at one-GPU scale (1024 PMUTs with 10
modes each; primary 128x128x8 hexes N = 4, secondary 96^3 hexes N = 3 behind
a non-conforming 4:3 interface; 32,822,146 unique DOFs), FP32 state and
operators, FP64 modal ODEs and traces.  A step is one pass of the whole hot
path: stiffness + interface residual + lumped-mass update for both bricks,
PMUT sampling / modal ODE / face force, receiver traces, interface fluxes.

Prints ONE JSON line (metric DOF-updates/s, whole job, inputs resident in HBM).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
STIFF_SOURCES = ["stiff_kernel.h", "stiff_f32_lo.hip", "stiff_f32_hi.hip"]
COUNTERS = os.path.join(ROOT, "profiles", "k_stiff_config3_fp32_hbm_counters.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(rows, zchunk):
    """HBM bytes per step of the two stiffness launches from the committed
    FETCH_SIZE / WRITE_SIZE passes, if the kernel sources and tile shape are
    still the ones those counters were taken with; else None."""
    import hashlib
    if (rows, zchunk) != (2, 33) or not os.path.exists(COUNTERS):
        return None
    h = hashlib.sha256()
    for f in STIFF_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_06267_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    fields = {}
    with open(COUNTERS) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_step", "stiff_source_sha256"):
                k, v = line.split(":", 1)
                fields[k] = v.strip()
    if fields.get("stiff_source_sha256") != h.hexdigest():
        return None
    return float(fields["traffic_bytes_per_step"])


def cpu_baseline(wl, steps):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload
    (the first `steps` steps of config 3), on all host cores."""
    from oracle import ref
    from paper_2603_06267_amd import workloads as W
    o = ref.from_workload(wl, shape_fn=W.shape_fn(wl))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    dofs = W.unique_dofs(wl)
    return {"value": dofs * steps / dt, "unit": "DOF-updates/s", "cores": ref.num_threads(), "kind": "oracle",
            "sample": f"{steps} steps of the same config-3 workload (FP64 oracle, {dt:.1f} s)"}


def run_gpu(wl, precision, steps, warmup, graphs, rows, zchunk):
    import torch
    from paper_2603_06267_amd import solver, workloads as W
    g = solver.from_workload(wl, precision=precision, n_steps=steps + warmup, shape_fn=W.shape_fn(wl),
                             device="cuda:0", bind=False)
    g.set_option(2, rows)
    g.set_option(3, zchunk)
    g.bind()
    stream = torch.cuda.current_stream()
    g.set_option(1, 1 if graphs else 0)
    g.step(warmup)
    torch.cuda.synchronize()
    # timed region: per-kernel HIP events on the stepping stream
    g.set_option(5, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = g.kernel_times()
    g.set_option(5, 0)
    # a second timed pass of graph replays (no events), same number of steps
    gg = solver.from_workload(wl, precision=precision, n_steps=steps + warmup, shape_fn=W.shape_fn(wl),
                              device="cuda:0", bind=False)
    gg.set_option(2, rows)
    gg.set_option(3, zchunk)
    gg.bind()
    gg.set_option(1, 1 if graphs else 0)
    gg.step(warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gg.step(steps)
    torch.cuda.synchronize()
    el_graph = time.perf_counter() - t1
    tr = gg.read_traces()
    finite = bool(np.isfinite(tr).all()) and not gg.nonfinite()
    return el, el_graph, kt, finite


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--rows", type=int, default=2)
    ap.add_argument("--zchunk", type=int, default=33)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 instantiation")
    ap.add_argument("--direct", action="store_true",
                    help="direct kernel launches instead of hipGraph replay (for counter collection)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported (the multi-GPU slab "
              "decomposition is a design only)", file=sys.stderr)
        sys.exit(2)

    from paper_2603_06267_amd import workloads as W
    wl = W.config3(steps=args.steps + args.warmup)
    dofs = W.unique_dofs(wl)
    n0 = int(np.prod([wl["domains"][0]["N"] * e + 1 for e in wl["domains"][0]["ne"]]))
    n1 = dofs - n0

    log(f"config 3: {dofs} unique DOFs ({W.element_local_dofs(wl)} element-local); FP32 run, "
        f"{args.warmup} warmup + {args.steps} timed steps")
    el, el_graph, kt, finite = run_gpu(wl, 32, args.steps, args.warmup, not args.direct, args.rows, args.zchunk)
    log(f"  timed (events): {el * 1e3 / args.steps:.4f} ms/step; graph replay: {el_graph * 1e3 / args.steps:.4f} "
        f"ms/step; kernels ms: stiff {kt[0]:.4f} face {kt[1]:.4f} flux {kt[2]:.4f}")
    best = min(el, el_graph)
    value = dofs * args.steps / best
    # algorithmic bytes per step of the stiffness launches (both bricks): read
    # p^n and p^{n-1}, write p^{n+1}, 4 bytes each per unique DOF.  The FP32
    # increment form moves 16 B per DOF by design (p and p^n - p^{n-1}).
    bytes_per_step = 12.0 * (n0 + n1)
    achieved = bytes_per_step / (kt[0] * 1e-3) / 1e9
    traffic = measured_traffic(args.rows, args.zchunk)
    out = {
        "metric": "DOF-updates/s",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "config3-large-array: 1024 PMUTs x 10 modes, primary 128x128x8 hexes N=4 + "
                               "secondary 96^3 hexes N=3, 4:3 non-conforming interface, FP32 state / FP64 ODE",
                   "unique_dofs": dofs, "element_local_dofs": W.element_local_dofs(wl),
                   "parallelism": "single GPU",
                   "timed_with": ("direct" if args.direct else "graph") + (" replay" if el_graph <= el else " + events")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "k_stiff, both bricks per step (12 B per unique DOF algorithmic; "
                               "traffic = measured HBM bytes per step)",
                     "moved_GBs": None if traffic is None else traffic / (kt[0] * 1e-3) / 1e9},
        "kernel_ms": {"stiff": kt[0], "face": kt[1], "flux": kt[2]},
        "finite": finite,
    }
    if not args.no_fp64:
        log("FP64 instantiation ...")
        el64, elg64, kt64, fin64 = run_gpu(wl, 64, args.steps, args.warmup, not args.direct, 1, args.zchunk)
        out["fp64"] = {"value": dofs * args.steps / min(el64, elg64), "unit": "DOF-updates/s",
                       "stiff_ms": kt64[0], "achieved_GBs": 24.0 * (n0 + n1) / (kt64[0] * 1e-3) / 1e9,
                       "frac": 24.0 * (n0 + n1) / (kt64[0] * 1e-3) / 1e9 / PEAK_HBM_GBS}
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        wl_cpu = W.config3(steps=args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(wl_cpu, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
