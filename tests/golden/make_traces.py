"""Writes the FP64 oracle's receiver traces of a benchmark workload to
tests/golden/config<N>_traces.npz:

- config 1: the cube with one PMUT (8 receivers), 1,000 steps;
- config 2: the two-domain array with 16 PMUTs and a 2:1 interface
  (64 receivers), 2,000 steps;
- config 3: the large array (1024 PMUTs, primary 128x128x8 hexes N = 4,
  secondary 96^3 hexes N = 3, 4:3 non-nested interface, beam steered 20
  degrees, 64 receivers), 5,000 steps; about two hours on seven host cores;
- config 4 (batched workload): scenario 0 of the cube with a 4x4 PMUT array
  and the highest-order uneven mesh (24x24x8 hexes, N = 6), 512 steps each,
  as config4base_traces.npz and config4mesh15_traces.npz;
- mapped: the large array's PMUT brick meshed by trilinear hexahedra whose
  edges follow every disc (128x128x8 hexes, N = 4, 1024 PMUTs), 1,000
  steps, as configmapped_traces.npz; about ten minutes on eight cores.

Only the oracle (oracle/ref.py, oracle/pmdg_ref.c) and the seeded input
generators (paper_2603_06267_amd/workloads.py) are used.  The run is the time
loop of Algorithm 1 in its synchronised reading, Sec. 3.1.  It is done in
chunks; with --ckpt-dir each chunk is followed by a checkpoint of the whole
oracle state there, so an interrupted run resumes where it stopped.

    python tests/golden/make_traces.py --config {1,2,3,4,mapped} [--steps 5000] [--chunk 250]
        [--ckpt-dir DIR]

Each stored file holds the traces [R x steps] (trace column n is time
(n+1) dt), the oracle's dt, the workload key (SHA-256 of every input array)
and the thread count.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ref  # noqa: E402
from paper_2603_06267_amd import workloads as W  # noqa: E402

STEPS = {"1": 1000, "2": 2000, "3": 5000, "4": 512, "mapped": 1000}


def golden_path(config):
    return os.path.join(HERE, f"config{config}_traces.npz")


def run(wl, steps, chunk, ckpt, tag):
    """Oracle traces [R x steps] of scenario 0 of a workload, in chunks, with
    an optional checkpoint file per chunk; returns (traces, dt, loop seconds)."""
    t0 = time.time()
    o = ref.from_workload(wl, shape_fn=W.shape_fn(wl))
    print(f"{tag}: oracle set up in {time.time() - t0:.1f} s: {o.n} nodes, dt = {o.dt!r}, "
          f"{ref.num_threads()} threads", flush=True)
    traces = np.zeros((o.R, steps))
    done = 0
    if ckpt is not None and os.path.exists(ckpt):
        z = np.load(ckpt)
        done = int(z["done"])
        traces[:, :done] = z["traces"][:, :done]
        o.set_state(p=z["p"], pd=z["pd"], pdd=z["pdd"], q=z["q"], qd=z["qd"], qdd=z["qdd"], nstep=done)
        print(f"resumed at step {done}", flush=True)
    t_loop = 0.0
    while done < steps:
        n = min(chunk, steps - done)
        t1 = time.time()
        traces[:, done:done + n] = o.step(n)
        t_loop += time.time() - t1
        done += n
        print(f"{tag} step {done}/{steps}: {time.time() - t1:.1f} s for {n} steps, "
              f"max |trace| {np.abs(traces[:, :done]).max():.4e}", flush=True)
        if ckpt is not None:
            st = o.get_state()
            assert st["nstep"] == done
            np.savez(ckpt + ".tmp.npz", done=done, traces=traces, p=st["p"], pd=st["pd"],
                     pdd=st["pdd"], q=st["q"], qd=st["qd"], qdd=st["qdd"])
            os.replace(ckpt + ".tmp.npz", ckpt)
    return traces, o.dt, t_loop


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", choices=tuple(STEPS), default="3")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--ckpt-dir", default=None)
    a = ap.parse_args()
    steps = a.steps or STEPS[a.config]
    if a.config == "4":
        # the batched workload: scenario 0 of the 4x4-PMUT cube and the
        # highest-order uneven mesh (24x24x8 hexes, N = 6)
        c4 = W.config4()
        jobs = [("4base", dict(c4["scenarios"], steps=steps)), ("4mesh15", dict(c4["meshes"][15], steps=steps))]
    elif a.config == "mapped":
        jobs = [("mapped", W.mapped_array(steps=steps))]
    else:
        jobs = [(a.config, dict(W.CONFIGS[int(a.config)](), steps=steps))]
    for tag, wl in jobs:
        key = W.workload_key(wl)
        ck = None
        if a.ckpt_dir:
            os.makedirs(a.ckpt_dir, exist_ok=True)
            ck = os.path.join(a.ckpt_dir, f"config{tag}_{key[:16]}.npz")
        traces, dt, t_loop = run(wl, steps, a.chunk, ck, tag)
        out = golden_path(tag)
        np.savez_compressed(out, traces=traces, dt=np.float64(dt), key=np.array(key),
                            steps=np.int64(steps), threads=np.int64(ref.num_threads()),
                            loop_seconds=np.float64(t_loop))
        print(f"wrote {out}: traces {traces.shape}, key {key[:16]}", flush=True)


if __name__ == "__main__":
    main()
