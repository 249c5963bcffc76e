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
# the kernel sources and the host code that picks their launch tiles
STIFF_SOURCES = ["stiff_kernel.h", "stiff_f32_lo.hip", "stiff_f32_hi.hip", "pmutdg.hip"]
COUNTERS = os.path.join(ROOT, "profiles", "k_stiff_config3_fp32_hbm_counters.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(rows, zchunk):
    """HBM bytes per step of the two stiffness launches from the committed
    FETCH_SIZE / WRITE_SIZE passes, if the kernel sources and tile shape are
    still the ones those counters were taken with; else None."""
    import hashlib
    if (rows, zchunk) != (0, 73) or not os.path.exists(COUNTERS):
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


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def golden_traces(config, wl):
    """FP64 oracle traces of a workload stored by tests/golden/make_traces.py
    (written by the oracle on the host), or None when absent or when they
    belong to other inputs."""
    from paper_2603_06267_amd import workloads as W
    path = os.path.join(GOLDEN_DIR, f"config{config}_traces.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    if str(z["key"]) != W.workload_key(wl):
        return None
    return z["traces"]


def trace_error(tg, to):
    """Relative L2 of GPU traces [R x n] against the oracle's over their
    common steps: all receivers together, and the largest receiver by
    receiver (each against max(its norm, 1% of the loudest))."""
    if to is None:
        return None
    n = min(tg.shape[-1], to.shape[-1])
    a, b = tg[:, :n], to[:, :n]
    nr = np.linalg.norm(b, axis=1)
    per = np.linalg.norm(a - b, axis=1) / np.maximum(nr, 0.01 * nr.max())
    return {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)), "per_receiver_max": float(per.max()),
            "steps": int(n)}


def trace_leg():
    """The large-array workload over its full 5,000 steps in the benchmark's
    launch configuration, FP32 and FP64, against the stored oracle traces."""
    import torch
    from paper_2603_06267_amd import solver, workloads as W
    wl = W.config3()
    to = golden_traces(3, wl)
    if to is None:
        return None
    out = {"reference": "FP64 CPU oracle, tests/golden/config3_traces.npz", "steps": int(to.shape[1])}
    for prec in (32, 64):
        g = solver.from_workload(wl, precision=prec, n_steps=to.shape[1], shape_fn=W.shape_fn(wl),
                                 device="cuda:0")
        g.step(to.shape[1])
        torch.cuda.synchronize()
        out[f"fp{prec}"] = trace_error(g.read_traces()[0], to)
        g.close()
    return out


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
    cores = ref.num_threads()
    # the same oracle on one thread, for one step of the same state
    ref.set_threads(1)
    try:
        t1 = time.perf_counter()
        o.step(1)
        dt1 = time.perf_counter() - t1
    finally:
        ref.set_threads(cores)
    return {"value": dofs * steps / dt, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} steps of the same config-3 workload (FP64 oracle, {dt:.1f} s)",
            "single_thread": {"value": dofs / dt1, "unit": "DOF-updates/s", "cores": 1,
                              "sample": f"step {steps + 1} of the same run on one thread ({dt1:.1f} s)"}}


def run_gpu(wl, precision, steps, warmup, graphs, rows, zchunk, tblock=1, overlap=None):
    import torch
    from paper_2603_06267_amd import solver, workloads as W
    g = solver.from_workload(wl, precision=precision, n_steps=steps + warmup, shape_fn=W.shape_fn(wl),
                             device="cuda:0", bind=False)
    g.set_option(2, rows)
    g.set_option(3, zchunk)
    g.set_option(9, tblock)
    if overlap is not None:
        g.set_option(10, overlap)
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
    gg.set_option(9, tblock)
    if overlap is not None:
        gg.set_option(10, overlap)
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
    run_gpu.traces = tr
    run_gpu.resident = gg.resident()
    return el, el_graph, kt, finite


def scenarios_leg(steps, warmup, rows, zchunk, S=4):
    """The large-array workload with S drive scenarios in one solver (beam
    steered to 20, 0, -20 and 40 degrees): S times the working set, well
    beyond the 256 MB last-level cache, so its rate cannot lean on that
    cache.  Same FP32 kernels, one launch per brick per step for all S."""
    import math
    from paper_2603_06267_amd import workloads as W
    wl = W.config3(steps=steps + warmup)
    ctr = np.asarray(wl["pmuts"]["centers"], dtype=np.float64)
    f = float(np.asarray(wl["drive"]["freq"]).reshape(-1)[0])
    angles = [20.0, 0.0, -20.0, 40.0][:S]
    phase = np.stack([2 * math.pi * f * ctr[:, 0] * math.sin(math.radians(a)) / W.C_WATER for a in angles])
    wl["drive"] = dict(wl["drive"], amp=np.ones((S, len(ctr))), phase=phase, freq=np.full(S, f))
    el, el_graph, kt, finite = run_gpu(wl, 32, steps, warmup, True, rows, zchunk)
    err = trace_error(run_gpu.traces[0], golden_traces(3, W.config3()))
    dofs = W.unique_dofs(wl)
    return {"scenarios": S, "trace_error_scenario0": err,
            "value": S * dofs * steps / min(el, el_graph), "unit": "DOF-updates/s",
            "ms_per_step": min(el, el_graph) * 1e3 / steps, "stiff_ms": kt[0],
            "achieved_GBs": 12.0 * S * dofs / (kt[0] * 1e-3) / 1e9,
            "frac": 12.0 * S * dofs / (kt[0] * 1e-3) / 1e9 / PEAK_HBM_GBS, "finite": finite}


def pml_workload(steps):
    """The large-array workload with perfectly matched layers in front of
    absorbing faces: 1 mm (3 coarse elements) on the secondary's side walls
    and top, 0.5 mm (2 fine elements) on the primary's side walls."""
    from paper_2603_06267_amd import workloads as W
    wl = W.config3(steps=steps)
    prim, sec = wl["domains"]
    prim = dict(prim, absorbing=0b001111, pml={"ell": [0.5, 0.5, 0.5, 0.5, 0.0, 0.0], "R": 1e-4})
    sec = dict(sec, absorbing=0b101111, pml={"ell": [1.0, 1.0, 1.0, 1.0, 0.0, 1.0], "R": 1e-4})
    return dict(wl, domains=[prim, sec])


def pml_leg(steps=200, warmup=10):
    """Rate of the large-array workload with matched layers (graph replay),
    the stiffness-plus-layer time per step, and the share of DOFs inside the
    layers' elements."""
    from paper_2603_06267_amd import workloads as W
    wl = pml_workload(steps + warmup)
    dofs = W.unique_dofs(wl)
    el, el_graph, kt, finite = run_gpu(wl, 32, steps, warmup, True, 0, 73)
    layer = 0
    for d in wl["domains"]:
        N, ne = d["N"], d["ne"]
        h = [(d["x1"][a] - d["x0"][a]) / ne[a] for a in range(3)]
        ell = d["pml"]["ell"]
        # nodes outside the layers' elements, per axis: the nodes of the
        # elements between the layers, less the face node shared with a layer
        free = [N * (ne[a] - round(ell[2 * a] / h[a]) - round(ell[2 * a + 1] / h[a])) + 1
                - (ell[2 * a] > 0) - (ell[2 * a + 1] > 0) for a in range(3)]
        layer += int(np.prod([N * e + 1 for e in ne])) - int(np.prod([max(v, 0) for v in free]))
    return {"workload": "config3 with matched layers: secondary side walls and top 1 mm, primary side walls "
                        "0.5 mm, absorbing outer faces", "unique_dofs": dofs, "layer_dofs": layer,
            "value": dofs * steps / min(el, el_graph), "unit": "DOF-updates/s",
            "ms_per_step": min(el, el_graph) * 1e3 / steps, "stiff_and_layer_ms": kt[0], "finite": finite}


def mapped_leg(steps=200, warmup=10):
    """The large array's PMUT brick meshed by trilinear hexahedra whose edges
    follow every disc (128x128x8 hexes, N = 4, 1024 PMUTs): rate with graph
    replay, the time of the two element-path launches per step against the
    bytes an update must move (read p, the increment X and the inverse mass,
    write p and X: 20 B per DOF, plus 96 B of corner offsets per element),
    and the trace error of a 1,000-step run against the oracle's stored
    traces."""
    from paper_2603_06267_amd import solver, workloads as W
    wl = W.mapped_array(steps=steps + warmup)
    dofs = W.unique_dofs(wl)
    d = wl["domains"][0]
    nel = int(np.prod(d["ne"]))
    n3 = (d["N"] + 1) ** 3
    el, el_graph, kt, finite = run_gpu(wl, 32, steps, warmup, True, 0, 73)
    alg = 20.0 * dofs + 96.0 * nel
    # the element residuals go through HBM once each way
    design = alg + 4.0 * dofs + 2 * 4.0 * nel * n3
    full = W.mapped_array()
    to = golden_traces("mapped", full)
    terr = None
    if to is not None:
        g = solver.from_workload(full, precision=32, shape_fn=W.shape_fn(full), device="cuda:0")
        g.step(full["steps"])
        terr = trace_error(g.read_traces()[0], to)
        g.close()
    return {"workload": "large-array PMUT brick, 128x128x8 trilinear hexes N=4 with edges on every disc, "
                        "1024 PMUTs", "unique_dofs": dofs, "elements": nel,
            "value": dofs * steps / min(el, el_graph), "unit": "DOF-updates/s",
            "ms_per_step": min(el, el_graph) * 1e3 / steps, "element_path_ms": kt[0],
            "roofline": {"bound": "hbm", "algorithmic_bytes": alg, "design_bytes": design,
                         "achieved": alg / (kt[0] * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": alg / (kt[0] * 1e-3) / 1e9 / PEAK_HBM_GBS},
            "finite": finite, "trace_error": terr}


def matching_leg(repeats=5):
    """Face matching of Sec. 5, Algorithm 3, on the large array's interface
    (16,384 fine faces, 5 x 5 Gauss points each, against 9,216 coarse faces),
    as bricks and with both sides warped: GPU time per call (HIP events) and
    the oracle's single-thread rate on a sample of 64 fine faces."""
    import torch
    from oracle import ref
    from paper_2603_06267_amd import matching as M, workloads as W
    wl = W.config3(steps=1)
    prim, sec = wl["domains"]
    out = {"fine_faces": prim["ne"][0] * prim["ne"][1], "coarse_faces": sec["ne"][0] * sec["ne"][1], "nq": 5}
    rng = np.random.default_rng(5)

    def warp(dom, amp=0.25):
        V = W.brick_vertices(dom)
        x0, x1 = np.asarray(dom["x0"]), np.asarray(dom["x1"])
        h = (x1 - x0) / np.asarray(dom["ne"])
        side = np.any(np.abs(V[:, :2] - x0[:2]) < 1e-12, axis=1) | np.any(np.abs(V[:, :2] - x1[:2]) < 1e-12, axis=1)
        V[~side, :2] += amp * h[:2] * rng.uniform(-1, 1, size=((~side).sum(), 2))
        return V

    for name, Vf, Vc in (("bricks", W.brick_vertices(prim), W.brick_vertices(sec)),
                         ("warped", warp(prim), warp(sec))):
        fine = M.layer_hexes(Vf, prim["ne"], prim["ne"][2] - 1)
        coarse = M.layer_hexes(Vc, sec["ne"], 0)
        ff, cf = np.full(len(fine), 5), np.full(len(coarse), 4)
        e, x, u = M.match_faces(5, fine, ff, coarse, cf)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(repeats):
            e, x, u = M.match_faces(5, fine, ff, coarse, cf)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / repeats
        npts = len(fine) * 25
        sample = np.sort(rng.choice(len(fine), size=64, replace=False))
        c0 = time.perf_counter()
        eo, xo, uo = ref.match_faces(5, fine[sample], ff[sample], coarse, cf)
        cpu = time.perf_counter() - c0
        pts = (sample[:, None] * 25 + np.arange(25)[None, :]).ravel()
        en = e.cpu().numpy()
        out[name] = {"points": npts, "gpu_ms": ms, "gpu_points_per_s": npts / (ms * 1e-3),
                     "unmatched": int(u.cpu().numpy()[0]),
                     "oracle_points_per_s": len(pts) / cpu, "oracle_threads": 1,
                     "sample_agrees": bool(np.array_equal(en[pts], eo))}
    return out


def resident_leg(steps=512):
    """Many drive scenarios of the batch cube (4x4 PMUTs, 4,913 nodes, N = 4)
    in one solver: the LDS-resident path (one workgroup per scenario, whole
    steps per launch) against the tiled path replayed as hipGraphs, for the
    64 scenarios of the batched workload and the 4,096 of the surrogate's
    data set; scenarios per second over `steps` steps each, and the trace
    error of scenario 0 of the 64 against the oracle's stored traces."""
    import torch
    from paper_2603_06267_amd import _lib, solver, workloads as W
    out = {}
    for name, wl in (("scenarios64", W.config4()["scenarios"]), ("scenarios4096", W.config5()["scenarios"])):
        S = np.asarray(wl["drive"]["amp"]).shape[0]
        wl = dict(wl, steps=steps)
        rates = {}
        for mode in (1, 0):
            g = solver.from_workload(wl, precision=32, n_steps=steps + 8, shape_fn=W.shape_fn(wl), device="cuda:0",
                                     bind=False)
            g.set_option(_lib.OPT_RESIDENT, mode)
            g.bind()
            g.step(8)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            rates["resident" if mode else "tiled"] = {"scenarios_per_s": S / el, "ms_per_step": el * 1e3 / steps,
                                                      "path_resident": g.resident()}
            if mode and name == "scenarios64":
                to = golden_traces("4base", dict(W.config4()["scenarios"], steps=512))
                rates["resident"]["trace_error"] = trace_error(g.read_traces()[0], to)
            g.close()
        rates["scenarios"] = S
        rates["unique_dofs"] = W.unique_dofs(wl)
        rates["speedup"] = rates["resident"]["scenarios_per_s"] / rates["tiled"]["scenarios_per_s"]
        out[name] = rates
    return out


def small_configs_leg(steps=400, warmup=20):
    """DOF-updates/s of the small workloads (the config-1 cube and the
    config-2 two-domain array), FP32 and FP64, hipGraph replay: latency-bound
    launches, reported as rates only."""
    from paper_2603_06267_amd import workloads as W
    out = {}
    for cfg, name, wl in ((1, "config1", W.config1()), (2, "config2", W.config2())):
        wl = dict(wl, steps=steps + warmup)
        dofs = W.unique_dofs(wl)
        to = golden_traces(cfg, wl)
        for prec in (32, 64):
            # automatic tiles; config 1 in FP32 fits the LDS-resident path
            el, el_graph, kt, finite = run_gpu(wl, prec, steps, warmup, True, 0, -1)
            out[f"{name}_fp{prec}"] = {"unique_dofs": dofs, "value": dofs * steps / min(el, el_graph),
                                       "ms_per_step": min(el, el_graph) * 1e3 / steps, "finite": finite,
                                       "resident": run_gpu.resident,
                                       "trace_error": trace_error(run_gpu.traces[0], to)}
    return out


def batched_leg(steps=512):
    """Batched form on the batch workload (64 drive scenarios of the cube with
    a 4x4 PMUT array + 16 uneven single-brick meshes, orders 3..6): one
    persistent launch sequence per step for all of them, against the same 80
    runs stepped one solver at a time (both as hipGraph replays, steps only)."""
    import torch
    from paper_2603_06267_amd import batch as B, solver, workloads as W
    c4 = W.config4()
    wls = [c4["scenarios"]] + c4["meshes"]
    sfs = [W.shape_fn(w) for w in wls]
    tuner = B.TileTuner(candidates=[(1, 17), (2, 17), (2, 33), (1, 0), (2, 0)])
    t0 = time.perf_counter()
    b = B.build_batch(wls, shape_fns=sfs, tuner=tuner, n_steps=steps)
    setup = time.perf_counter() - t0
    b.step(8)
    torch.cuda.synchronize()
    t = time.perf_counter()
    b.step(steps - 8)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    err = {"scenario0": trace_error(b.solvers[0].read_traces()[0], golden_traces("4base", wls[0])),
           "mesh15": trace_error(b.solvers[16].read_traces()[0], golden_traces("4mesh15", wls[16]))}
    nsc = sum(len(w["drive"]["amp"]) for w in wls)
    singles = []
    for w, sf in zip(wls, sfs):
        for sc in range(len(w["drive"]["amp"])):
            singles.append(solver.from_workload(w, precision=32, n_steps=steps, scenarios=[sc], shape_fn=sf))
    for s1 in singles:
        s1.step(8)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for s1 in singles:
        s1.step(steps - 8)
    torch.cuda.synchronize()
    el2 = time.perf_counter() - t
    frac = (steps - 8) / steps
    return {"workload": "64 scenarios (cube, 4x4 PMUTs, 3 modes) + 16 meshes 8x8x4..24x24x8 N=3..6, 512 steps",
            "scenarios": nsc, "batched_scenarios_per_s": nsc * frac / el, "loop_scenarios_per_s": nsc * frac / el2,
            "speedup": el2 / el, "trace_error": err, "setup_and_tuning_s": setup, "tiles": {k: v["best"] for k, v in tuner.cache.items()}}


def surrogate_leg(runs, steps, log, batch=256, lr=1e-3, method="linear"):
    """Surrogate form: data from the GPU solver, a two-member network trained
    on it (method "linear": the library's least-squares fit, each member on
    its own half of the training rows; "adam": He initialisation and the
    library's BF16-MFMA forward / backward / Adam kernels), split-conformal
    calibration, then inference with solver fallback at 2% relative L2 on the
    256 held-out test scenarios and on a fresh batch of 1024, against the
    plain solver one scenario at a time and batched."""
    import torch
    from paper_2603_06267_amd import mlp as MLPmod, surrogate as S, workloads as W
    c5 = W.config5()
    F = c5["features"]
    if runs > len(F):
        rng = np.random.default_rng(W.SEED0 + 55)
        ph, fr, am = W.scenario_params(rng, runs - len(F))
        F = np.concatenate([F, np.concatenate([ph, fr[:, None], am[:, None]], 1)])
    t0 = time.perf_counter()
    T = S.solve(F)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    U = torch.as_tensor(F.astype(np.float32), device="cuda")
    train = np.concatenate([np.arange(3584), np.arange(4096, len(F))])
    cal, test = np.arange(3584, 3840), np.arange(3840, 4096)
    if method == "linear":
        sur = S.Surrogate(n_members=2, n_cos=S.N_COS)
        t_train = sur.fit_linear(U, T, train, npairs=S.N_PAIRS, rank=S.RANK)
        how = {"method": "least-squares fit (pmdg_mlp_fit_linear), members on disjoint halves",
               "input_columns": len(sur.columns), "rank": S.RANK, "pairs": S.N_PAIRS}
    else:
        sur = S.Surrogate(n_members=2, n_fourier=8)
        t_train = sur.fit(U, T, train, steps=steps, batch=batch, lr=lr, log=log, log_every=max(1, steps // 4))
        how = {"method": "Adam from He initialisation", "train_steps_per_member": steps, "minibatch": batch,
               "lr": lr, "input_columns": len(sur.columns)}
    scale = sur.calibrate(U, T, cal)
    err, spread = sur.errors(U, T, test)
    est = sur.estimate(spread)

    def delivered(out, rows_dev, Tref):
        return MLPmod.row_errors(out, Tref, rows_dev).cpu().numpy()

    # inference with fallback on the 256 test scenarios at the 2% tolerance
    # and, for context, looser ones
    test_dev = torch.as_tensor(test.astype(np.int32), device="cuda")
    by_tol = {}
    for tol in (S.TOL, 0.05, 0.1):
        sur.infer(F[test[:8]], tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, mask, _ = sur.infer(F[test], tol=tol)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d = delivered(out, test_dev, T)
        by_tol[f"{tol:g}"] = {"routed_to_solver": float(mask.mean()), "scenarios_per_s": len(test) / el,
                              "delivered_share_above_tol": float(np.mean(d > tol))}
        if tol == S.TOL:
            derr, mask2 = d, mask
    # a fresh inference batch of 1024 scenarios (new seed): the pipeline
    # against the plain solver on the same scenarios
    rng = np.random.default_rng(W.SEED0 + 77)
    ph, fr, am = W.scenario_params(rng, 1024)
    Fb = np.concatenate([ph, fr[:, None], am[:, None]], 1)
    # steady state: one untimed call of each first, so the solvers the calls
    # restart (one per scenario-slot count) exist before the timed ones
    S.solve(Fb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Tb = S.solve(Fb)
    torch.cuda.synchronize()
    batched = 1024 / (time.perf_counter() - t0)
    sur.infer(Fb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outb, maskb, _ = sur.infer(Fb)
    torch.cuda.synchronize()
    pipeline = 1024 / (time.perf_counter() - t0)
    db = delivered(outb, None, Tb)
    # network alone, batch 1024
    Ub = torch.as_tensor(Fb.astype(np.float32), device="cuda")
    for _ in range(3):
        sur.predict(Ub)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        sur.predict(Ub)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t0) / 10
    # the plain solver one scenario at a time (8 timed, after one untimed)
    S.solve(F[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(8):
        S.solve(F[r:r + 1])
    torch.cuda.synchronize()
    single = 8 / (time.perf_counter() - t0)
    return {"workload": f"cube with 4x4 PMUTs, 64 receivers x 512 samples; {len(F)} solver runs "
                        f"({len(train)} train, 256 calibration, 256 test); inference batch 1024 fresh scenarios",
            "training": how, "data_s": t_data, "train_s": t_train,
            "test_rel_l2_median": float(np.median(err)), "test_rel_l2_p90": float(np.quantile(err, 0.9)),
            "calibration_scale": scale, "coverage": float(np.mean(err <= est)),
            "certified_at_2pct": float(np.mean(est <= S.TOL)),
            "routed_to_solver": float(mask2.mean()), "delivered_rel_l2_median": float(np.median(derr)),
            "delivered_share_above_2pct": float(np.mean(derr > S.TOL)),
            "batch1024": {"routed_to_solver": float(maskb.mean()), "delivered_rel_l2_median": float(np.median(db)),
                          "delivered_share_above_2pct": float(np.mean(db > S.TOL)),
                          "pipeline_scenarios_per_s": pipeline, "solver_batched_scenarios_per_s": batched},
            "pipeline_scenarios_per_s": pipeline, "network_scenarios_per_s": 1024 / t_net,
            "solver_single_scenarios_per_s": single, "solver_batched_scenarios_per_s": batched,
            "gain_vs_single": pipeline / single, "gain_vs_batched": pipeline / batched, "by_tolerance": by_tol}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--rows", type=int, default=0, help="rows per wave of the stiffness tile (0: automatic)")
    ap.add_argument("--zchunk", type=int, default=73)
    ap.add_argument("--overlap", type=int, default=None, choices=(0, 1, 2, 3),
                    help="PMDG_OPT_OVERLAP for the large-array run (default: the library's)")
    ap.add_argument("--tblock", type=int, default=1, choices=(1, 2),
                    help="steps per stiffness pass (2: the fused two-step pass)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 instantiation")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-scenarios", action="store_true",
                    help="skip the large-array leg with 4 drive scenarios in one solver")
    ap.add_argument("--no-small", action="store_true", help="skip the small-workload rates")
    ap.add_argument("--no-pml", action="store_true", help="skip the large array with matched layers")
    ap.add_argument("--pml-only", action="store_true",
                    help="run only the large array with matched layers (direct launches, for counters)")
    ap.add_argument("--no-mapped", action="store_true",
                    help="skip the PMUT brick meshed by trilinear hexahedra and the face matching")
    ap.add_argument("--mapped-only", action="store_true",
                    help="run only the trilinear-hexahedron brick (direct launches with --direct, for counters)")
    ap.add_argument("--no-trace", action="store_true",
                    help="skip the full 5,000-step large-array runs compared with the oracle's traces")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-form leg")
    ap.add_argument("--surrogate-runs", type=int, default=4096)
    ap.add_argument("--surrogate-steps", type=int, default=3000)
    ap.add_argument("--surrogate-extended", action="store_true",
                    help="also train by Adam on the larger solver-generated data set")
    ap.add_argument("--no-surrogate-adam", action="store_true",
                    help="skip the network trained by Adam from He initialisation (for comparison)")
    ap.add_argument("--surrogate-extended-runs", type=int, default=65536)
    ap.add_argument("--surrogate-extended-steps", type=int, default=60000)
    ap.add_argument("--direct", action="store_true",
                    help="direct kernel launches instead of hipGraph replay (for counter collection)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported (the multi-GPU slab "
              "decomposition is a design only)", file=sys.stderr)
        sys.exit(2)

    from paper_2603_06267_amd import workloads as W
    if args.pml_only:
        wl = pml_workload(args.steps + args.warmup)
        el, el_graph, kt, finite = run_gpu(wl, 32, args.steps, args.warmup, not args.direct, 0, 73)
        print(json.dumps({"pml_only": True, "ms_per_step": min(el, el_graph) * 1e3 / args.steps,
                          "stiff_and_layer_ms": kt[0], "finite": finite}), flush=True)
        return
    if args.mapped_only:
        wl = W.mapped_array(steps=args.steps + args.warmup)
        el, el_graph, kt, finite = run_gpu(wl, 32, args.steps, args.warmup, not args.direct, 0, 73)
        print(json.dumps({"mapped_only": True, "ms_per_step": min(el, el_graph) * 1e3 / args.steps,
                          "element_path_ms": kt[0], "finite": finite}), flush=True)
        return
    wl = W.config3(steps=args.steps + args.warmup)
    dofs = W.unique_dofs(wl)
    n0 = int(np.prod([wl["domains"][0]["N"] * e + 1 for e in wl["domains"][0]["ne"]]))
    n1 = dofs - n0

    log(f"config 3: {dofs} unique DOFs ({W.element_local_dofs(wl)} element-local); FP32 run, "
        f"{args.warmup} warmup + {args.steps} timed steps")
    el, el_graph, kt, finite = run_gpu(wl, 32, args.steps, args.warmup, not args.direct, args.rows, args.zchunk,
                                       args.tblock, args.overlap)
    log(f"  timed (events): {el * 1e3 / args.steps:.4f} ms/step; graph replay: {el_graph * 1e3 / args.steps:.4f} "
        f"ms/step; kernels ms: stiff {kt[0]:.4f} face {kt[1]:.4f} flux {kt[2]:.4f}")
    main_err = trace_error(run_gpu.traces[0], golden_traces(3, W.config3()))
    best = min(el, el_graph)
    value = dofs * args.steps / best
    # algorithmic bytes per step of the stiffness launches (both bricks): read
    # p^n and p^{n-1}, write p^{n+1}, 4 bytes each per unique DOF.  The FP32
    # increment form moves 16 B per DOF by design (p and p^n - p^{n-1}).
    bytes_per_step = 12.0 * (n0 + n1)
    achieved = bytes_per_step / (kt[0] * 1e-3) / 1e9
    traffic = measured_traffic(args.rows, args.zchunk) if args.tblock == 1 else None
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
        "trace_error": main_err,
    }
    if not args.no_fp64:
        log("FP64 instantiation ...")
        el64, elg64, kt64, fin64 = run_gpu(wl, 64, args.steps, args.warmup, not args.direct, 1, args.zchunk)
        out["fp64"] = {"value": dofs * args.steps / min(el64, elg64), "unit": "DOF-updates/s",
                       "trace_error": trace_error(run_gpu.traces[0], golden_traces(3, W.config3())),
                       "stiff_ms": kt64[0], "achieved_GBs": 24.0 * (n0 + n1) / (kt64[0] * 1e-3) / 1e9,
                       "frac": 24.0 * (n0 + n1) / (kt64[0] * 1e-3) / 1e9 / PEAK_HBM_GBS}
    if not args.no_trace:
        log("large array, full run against the oracle's traces ...")
        out["trace_rel_l2"] = trace_leg()
    if not args.no_scenarios:
        log("large array x 4 scenarios ...")
        out["scenarios4"] = scenarios_leg(min(args.steps, 200), args.warmup, args.rows, args.zchunk)
    if not args.no_pml:
        log("large array with matched layers ...")
        out["pml"] = pml_leg()
    if not args.no_mapped:
        log("trilinear-hexahedron PMUT brick ...")
        out["mapped"] = mapped_leg()
        log("face matching (Algorithm 3) ...")
        out["matching"] = matching_leg()
    if not args.no_small:
        log("small workloads ...")
        out["small"] = small_configs_leg()
        log("LDS-resident scenarios ...")
        out["resident"] = resident_leg()
    if not args.no_batched:
        log("batched form ...")
        out["batched"] = batched_leg()
    if not args.no_surrogate:
        log("surrogate form ...")
        out["surrogate"] = surrogate_leg(args.surrogate_runs, args.surrogate_steps, log)
        if not args.no_surrogate_adam:
            log("surrogate form, network trained by Adam ...")
            out["surrogate_adam"] = surrogate_leg(args.surrogate_runs, args.surrogate_steps, log, method="adam")
        if args.surrogate_extended:
            log("surrogate form, Adam on the larger data set ...")
            out["surrogate_extended"] = surrogate_leg(args.surrogate_extended_runs, args.surrogate_extended_steps, log,
                                                      batch=512, lr=2e-3, method="adam")
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        wl_cpu = W.config3(steps=args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(wl_cpu, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
