"""Writes the FP64 oracle's receiver traces of the large-array workload
(1024 PMUTs, primary 128x128x8 hexes N = 4, secondary 96^3 hexes N = 3,
4:3 non-nested interface, beam steered 20 degrees, 64 receivers) to
tests/golden/config3_traces.npz.

Only the oracle (oracle/ref.py, oracle/pmdg_ref.c) and the seeded input
generators (paper_2603_06267_amd/workloads.py) are used.  The run is the time
loop of Algorithm 1 in its synchronised reading, Sec. 3.1; it takes about an
hour on eight host cores and is done in chunks, each followed by a
checkpoint of the whole oracle state in --ckpt-dir, so an interrupted run
resumes where it stopped.

    python tests/golden/make_config3_traces.py [--steps 5000] [--chunk 250]
        [--ckpt-dir DIR]

The stored file holds the traces [R x steps] (trace column n is time
(n+1) dt), the oracle's dt, the workload key (SHA-256 of every input array)
and the thread count.
"""
import argparse
import hashlib
import json
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

OUT = os.path.join(HERE, "config3_traces.npz")


def workload_key(wl):
    """SHA-256 over every input array of a workload description (domains,
    PMUT data, drive, receivers), so a changed generator invalidates the
    stored traces."""
    h = hashlib.sha256()
    h.update(json.dumps(wl["domains"], sort_keys=True).encode())
    h.update(json.dumps([wl.get("cfl"), wl.get("alpha")]).encode())
    for k in ("centers", "radius", "omega", "zeta", "eta", "scale"):
        h.update(np.ascontiguousarray(wl["pmuts"][k], dtype=np.float64).tobytes())
    dr = wl["drive"]
    for k in ("amp", "phase", "freq"):
        h.update(np.ascontiguousarray(dr[k], dtype=np.float64).tobytes())
    h.update(json.dumps([dr["ncyc"], dr.get("envelope", 0)]).encode())
    h.update(np.ascontiguousarray(wl["receivers"], dtype=np.float64).tobytes())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--ckpt-dir", default=None)
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()

    wl = W.config3(steps=a.steps)
    key = workload_key(wl)
    t0 = time.time()
    o = ref.from_workload(wl, shape_fn=W.shape_fn(wl))
    print(f"oracle set up in {time.time() - t0:.1f} s: {o.n} nodes, dt = {o.dt!r}, "
          f"{ref.num_threads()} threads", flush=True)

    traces = np.zeros((o.R, a.steps))
    done = 0
    ck = None
    if a.ckpt_dir:
        os.makedirs(a.ckpt_dir, exist_ok=True)
        ck = os.path.join(a.ckpt_dir, f"config3_{key[:16]}.npz")
        if os.path.exists(ck):
            z = np.load(ck)
            done = int(z["done"])
            traces[:, :done] = z["traces"][:, :done]
            o.set_state(p=z["p"], pd=z["pd"], pdd=z["pdd"], q=z["q"], qd=z["qd"], qdd=z["qdd"],
                        nstep=done)
            print(f"resumed at step {done}", flush=True)
    t_loop = 0.0
    while done < a.steps:
        n = min(a.chunk, a.steps - done)
        t1 = time.time()
        traces[:, done:done + n] = o.step(n)
        t_loop += time.time() - t1
        done += n
        print(f"step {done}/{a.steps}: {time.time() - t1:.1f} s for {n} steps, "
              f"max |trace| {np.abs(traces[:, :done]).max():.4e}", flush=True)
        if ck is not None:
            st = o.get_state()
            assert st["nstep"] == done
            np.savez(ck + ".tmp.npz", done=done, traces=traces, p=st["p"], pd=st["pd"],
                     pdd=st["pdd"], q=st["q"], qd=st["qd"], qdd=st["qdd"])
            os.replace(ck + ".tmp.npz", ck)
    np.savez_compressed(a.out, traces=traces, dt=np.float64(o.dt), key=np.array(key),
                        steps=np.int64(a.steps), threads=np.int64(ref.num_threads()),
                        loop_seconds=np.float64(t_loop))
    print(f"wrote {a.out}: traces {traces.shape}, key {key[:16]}", flush=True)


if __name__ == "__main__":
    main()
