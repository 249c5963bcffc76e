"""Surrogate form: a network trained on runs of the solver itself that maps a
PMUT array's drive parameters (16 per-PMUT phases, frequency, amplitude) to
its receiver traces (64 receivers x 512 samples), with a calibrated error
estimate and the solver as fallback.

  data       the GPU solver (FP32 state, FP64 modal ODE and traces) on the
             seeded scenarios of the surrogate data set, one batched launch
  network    18 drive parameters -> 512 -> 512 -> 512 -> 512 -> 32768, GELU,
             run by the library's BF16-MFMA kernels.  Each phase enters as
             the pair (cos, sin) (phases are angles), frequency and amplitude
             affinely, and each phase column also times a cosine series in
             frequency (N_COS terms): the solver is linear in each PMUT's
             drive, so the traces are a linear function of those products.
             Training: the least-squares fit of the library
             (pmdg_mlp_fit_linear) writes the network that computes the best
             rank-RANK linear map of the inputs; Adam on the library's forward
             / backward kernels (fit) remains available.  The output is scaled
             by the amplitude, since the solver's traces are exactly
             proportional to it
  estimate   a two-member ensemble (members fitted on disjoint halves of the
             training rows); its spread |y_1 - y_2| / |(y_1 + y_2) / 2|, scaled by the
             split-conformal quantile of (true error / spread) on a held-out
             calibration set, bounds the relative L2 error of the ensemble
             mean with the stated coverage
  fallback   scenarios whose estimate exceeds the tolerance (2% relative L2)
             are re-run by the solver; the solver's traces replace them

Host code here is control flow (minibatch order, learning-rate schedule,
quantiles over a few hundred numbers); every array operation of the path runs
in libpmutdg's kernels."""
import math
import time

import numpy as np

from . import mlp as _mlp
from . import solver as _solver
from . import workloads as W

HIDDEN = [512, 512, 512, 512]
N_OUT = 64 * 512
N_PMUT = 16
TOL = 0.02
# default network input and least-squares fit: cosine series of 24 terms in
# frequency times each phase column (770 inputs), rank 416 with the leading
# 96 directions passed as pairs (96 x 2 + 320 = 512 hidden units)
N_COS = 24
RANK = 416
N_PAIRS = 96


AMP_COL = N_PMUT + 1
FREQ_COL = N_PMUT
# drive frequencies of the data set, U[F_LO, F_LO + F_SPAN] MHz
F_LO, F_SPAN = 1.5, 1.5
# sampled trace length (512 steps of the cube's dt = 8.634 ns), for the
# frequency's Fourier columns
T_TRACE_US = 4.42


def input_columns(n_fourier=0, n_product=0, n_cos=0):
    """Embedding of the raw features [phase x16, frequency (MHz), amplitude]:
    each phase as (cos, sin) (phases are angles), frequency in [1.5, 3] and
    amplitude in [0.5, 1] mapped affinely onto [-1, 1], and optionally
    n_fourier pairs cos / sin(2 pi tau_j f), tau_j = j T / n_fourier, which give
    the network the oscillation of the traces with frequency at the sampled
    times.  n_product > 0 adds, for every phase column and j = 1 .. n_product,
    its products with cos / sin(2 pi tau_j f), tau_j = j T / n_product: the
    traces are linear in each PMUT's drive (A cos theta_k, A sin theta_k), so
    these products span their dependence on phase and frequency together,
    which a network would otherwise have to form from separate columns.
    n_cos > 0 adds the products of every phase column with the cosine series
    cos(pi j (f - F_LO) / F_SPAN), j = 1 .. n_cos - 1: over the data set's
    uniform frequencies these are orthogonal to one another and to the phase
    columns (condition number of the embedded rows about 3), so a linear
    least-squares map on them is well posed in FP32 and BF16."""
    cols = []
    for k in range(N_PMUT):
        cols += [(k, 1, 0.0, 1.0), (k, 2, 0.0, 1.0)]
    cols += [(FREQ_COL, 0, 2.25, 1.0 / 0.75), (AMP_COL, 0, 0.75, 4.0)]
    for j in range(1, n_fourier + 1):
        w = 2.0 * math.pi * j * T_TRACE_US / n_fourier
        cols += [(FREQ_COL, 1, 0.0, w), (FREQ_COL, 2, 0.0, w)]
    for k in range(N_PMUT):
        for op in (1, 2):
            for j in range(1, n_product + 1):
                w = 2.0 * math.pi * j * T_TRACE_US / n_product
                cols += [(k, op, 0.0, 1.0, FREQ_COL, 1, 0.0, w), (k, op, 0.0, 1.0, FREQ_COL, 2, 0.0, w)]
    for k in range(N_PMUT):
        for op in (1, 2):
            for j in range(1, n_cos):
                cols.append((k, op, 0.0, 1.0, FREQ_COL, 1, -math.pi * j * F_LO / F_SPAN, math.pi * j / F_SPAN))
    return cols


def drive_from_features(F):
    """Drive description of the solver for feature rows [phase x16, freq, amp]."""
    F = np.asarray(F, dtype=np.float64)
    return {"amp": np.repeat(F[:, 17:18], N_PMUT, axis=1), "phase": F[:, :N_PMUT].copy(), "freq": F[:, 16].copy(),
            "ncyc": 3.0, "envelope": 0}


# Bound solvers of the batch geometry, one per (device, steps, scenario
# slots): a solve restarts one and sets the new drive instead of building a
# solver again (the set-up costs more than the run for a few hundred
# scenarios).
_SOLVERS = {}


def _slots(n, max_scenarios):
    """Scenario slots for n rows: the next power of two from 64 (a few sizes
    serve every batch; spare slots repeat the first row)."""
    k = 64
    while k < n:
        k *= 2
    return min(k, max_scenarios)


def _cached_solver(S, steps, device):
    key = (str(device), steps, S)
    g = _SOLVERS.get(key)
    if g is None:
        base = W.batch_geometry()
        F0 = np.zeros((S, N_PMUT + 2))
        F0[:, N_PMUT], F0[:, N_PMUT + 1] = 2.0, 1.0
        wl = dict(base, drive=drive_from_features(F0))
        g = _solver.from_workload(wl, precision=32, n_steps=steps, shape_fn=W.shape_fn(base), device=device)
        _SOLVERS[key] = g
    return g


def clear_solver_cache():
    """Releases the cached solvers and their workspaces."""
    for g in _SOLVERS.values():
        g.close()
    _SOLVERS.clear()


def solve(F, steps=512, device="cuda", stream=None, max_scenarios=4096):
    """Runs the plain GPU solver for feature rows F; returns device FP32 traces
    [len(F), R * steps] (receiver-major).  Scenarios go in launches of at most
    max_scenarios, each on a cached solver restarted with the new drive."""
    import torch
    F = np.asarray(F, dtype=np.float64)
    out = []
    for i0 in range(0, len(F), max_scenarios):
        rows = F[i0:i0 + max_scenarios]
        n = len(rows)
        S = _slots(n, max_scenarios)
        g = _cached_solver(S, steps, device)
        if S > n:
            rows = np.concatenate([rows, np.repeat(rows[:1], S - n, axis=0)])
        dr = drive_from_features(rows)
        g.restart(stream)
        g.set_drive(dr["amp"], dr["phase"], dr["freq"], dr["ncyc"], dr["envelope"])
        g.step(steps, stream)
        tr = g.read_traces_device(32, stream)[:n]
        out.append(tr.reshape(n, -1))
    return torch.cat(out) if len(out) > 1 else out[0]


class Surrogate:
    def __init__(self, n_members=2, max_batch=1024, seed=0, device="cuda", n_fourier=0, hidden=None, n_out=N_OUT,
                 n_product=0, n_cos=0):
        self.columns = input_columns(n_fourier, n_product, n_cos)
        self.widths = [len(self.columns)] + list(hidden or HIDDEN) + [n_out]
        self.members = [_mlp.MLP(self.widths, max_batch=max_batch, device=device) for _ in range(n_members)]
        self.max_batch = max_batch
        self.device = device
        self.seed = seed
        self.scale = None
        self.out_scale = 1.0
        self.history = []

    # ---- training ---------------------------------------------------------
    def fit(self, U, T, train_idx, steps=3000, batch=256, lr=1e-3, lr_final=1e-5, log=None, log_every=500):
        """U [n, 18], T [n, n_out]: device FP32 tensors; train_idx: host ints.
        Each member: He initialisation from its own seed, its own minibatch
        order, Adam with a cosine learning-rate decay from lr to lr_final."""
        import torch
        tr = torch.as_tensor(np.asarray(train_idx).astype(np.int32), device=U.device)
        # RMS of the amplitude-normalised training traces
        self.members[0].set_io_map(N_PMUT + 2, self.columns, amp_col=AMP_COL)
        self.members[0].set_target_scale(U, T, tr, len(train_idx))
        self.out_scale = self.members[0].out_scale
        err = torch.empty(batch, dtype=torch.float32, device=U.device)
        nrm = torch.empty(batch, dtype=torch.float32, device=U.device)
        ntr = len(train_idx)
        t0 = time.perf_counter()
        for k, m in enumerate(self.members):
            rng = np.random.default_rng(self.seed + 1000 * k)
            m.set_io_map(N_PMUT + 2, self.columns, out_scale=self.out_scale, amp_col=AMP_COL)
            m.init_params(rng)
            per_epoch = ntr // batch
            perm = None
            for s in range(steps):
                if s % per_epoch == 0:
                    # one upload per epoch: the minibatches are views of it
                    order = np.asarray(train_idx)[rng.permutation(ntr)][:per_epoch * batch]
                    perm = torch.as_tensor(order.astype(np.int32), device=U.device)
                j = s % per_epoch
                idx = perm[j * batch:(j + 1) * batch]
                a = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * s / steps))
                m.train_step(U, T, idx, a, rowerr=err, rownorm=nrm)
                if log and (s % log_every == 0 or s == steps - 1):
                    rel = torch.sqrt(err / nrm).median().item()
                    self.history.append((k, s, rel))
                    log(f"member {k} step {s}: minibatch median rel L2 {rel:.4f} "
                        f"({time.perf_counter() - t0:.1f} s)")
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def fit_linear(self, U, T, train_idx, npairs=96, rank=416, ridge=0.0, finetune_steps=0, batch=256, lr=1e-5):
        """Least-squares training (pmdg_mlp_fit_linear): the training rows are
        split into disjoint parts by a seeded permutation, one per member, and
        each member is fitted on its own part, so that the members' spread
        reflects what the data leave undetermined.  finetune_steps > 0 then
        runs that many Adam steps per member on all training rows (cosine
        decay from lr)."""
        import torch
        t0 = time.perf_counter()
        rng = np.random.default_rng(self.seed)
        perm = np.asarray(train_idx)[rng.permutation(len(train_idx))]
        parts = np.array_split(perm, len(self.members))
        for m, part in zip(self.members, parts):
            m.set_io_map(N_PMUT + 2, self.columns, amp_col=AMP_COL)
            idx = torch.as_tensor(np.sort(part).astype(np.int32), device=U.device)
            m.fit_linear(U, T, idx, len(part), npairs, rank, ridge)
        self.out_scale = self.members[0].out_scale
        if finetune_steps > 0:
            err = torch.empty(batch, dtype=torch.float32, device=U.device)
            nrm = torch.empty(batch, dtype=torch.float32, device=U.device)
            ntr = len(train_idx)
            per_epoch = ntr // batch
            for k, m in enumerate(self.members):
                g = np.random.default_rng(self.seed + 1000 * k + 1)
                for s in range(finetune_steps):
                    if s % per_epoch == 0:
                        order = np.asarray(train_idx)[g.permutation(ntr)][:per_epoch * batch]
                        sel = torch.as_tensor(order.astype(np.int32), device=U.device)
                    j = s % per_epoch
                    a = 0.5 * lr * (1 + math.cos(math.pi * s / finetune_steps))
                    m.train_step(U, T, sel[j * batch:(j + 1) * batch], a, rowerr=err, rownorm=nrm)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # ---- inference --------------------------------------------------------
    def predict(self, U, idx=None, out=None, stream=None):
        """Ensemble mean [B, n_out] and raw spread |y1 - y2| / |mean| per row."""
        import torch
        B = int(idx.shape[0]) if idx is not None else int(U.shape[0])
        assert B <= self.max_batch and B % 8 == 0
        ys = [m.forward(U, idx=idx, stream=stream) for m in self.members]
        if len(ys) == 1:
            return ys[0], torch.zeros(B, device=U.device)
        return _mlp.pair_combine(ys[0], ys[1], mean=ys[0] if out is None else out, stream=stream)

    def calibrate(self, U, T, cal_idx, coverage=0.95):
        """Split-conformal scale: the ceil((n + 1) coverage)-th smallest of
        (true relative error / spread) over the calibration rows."""
        import torch
        err, spread = self.errors(U, T, cal_idx)
        r = np.sort(err / np.maximum(spread, 1e-12))
        n = len(r)
        k = min(n - 1, int(math.ceil((n + 1) * coverage)) - 1)
        self.scale = float(r[k])
        return self.scale

    def errors(self, U, T, rows):
        """True relative L2 error of the ensemble mean and its spread, per row
        (host arrays); rows in batches of max_batch."""
        import torch
        errs, spreads = [], []
        rows = np.asarray(rows)
        for i0 in range(0, len(rows), self.max_batch):
            r = rows[i0:i0 + self.max_batch]
            pad = (-len(r)) % 8
            rr = np.concatenate([r, np.repeat(r[-1:], pad)]) if pad else r
            idx = torch.as_tensor(rr.astype(np.int32), device=U.device)
            mean, spread = self.predict(U, idx=idx)
            e = _mlp.row_errors(mean, T, idx)
            errs.append(e[:len(r)].cpu().numpy())
            spreads.append(spread[:len(r)].cpu().numpy())
        return np.concatenate(errs), np.concatenate(spreads)

    def estimate(self, spread):
        return self.scale * spread

    def infer(self, F, U=None, tol=TOL, stream=None):
        """Traces for feature rows F (host [B, 18], B <= max_batch, multiple
        of 8): ensemble mean where the calibrated estimate is <= tol, the
        solver's traces elsewhere.  Returns (device traces, host mask of rows
        sent to the solver, host estimates)."""
        import torch
        assert self.scale is not None, "calibrate first"
        if U is None:
            U = torch.as_tensor(np.asarray(F, dtype=np.float32), device=self.device)
        mean, spread = self.predict(U, stream=stream)
        est = (self.scale * spread).cpu().numpy()
        mask = est > tol
        if mask.any():
            rows = np.nonzero(mask)[0]
            sol = solve(np.asarray(F)[rows], stream=stream)
            _mlp.scatter_rows(sol, torch.as_tensor(rows.astype(np.int32), device=mean.device), mean, stream=stream)
        return mean, mask, est


def bench_network(n_infer=20, n_train=50, batch_infer=1024, batch_train=256, n_fourier=8, seed=0):
    """Times the network kernels alone on synthetic rows: inference passes of
    batch_infer rows and training steps of batch_train rows (ms each)."""
    import torch
    from . import mlp as _m
    cols = input_columns(n_fourier)
    widths = [len(cols)] + HIDDEN + [N_OUT]
    m = _m.MLP(widths, max_batch=max(batch_infer, batch_train))
    m.set_io_map(N_PMUT + 2, cols, out_scale=0.3, amp_col=AMP_COL)
    rng = np.random.default_rng(seed)
    m.init_params(rng)
    n = 4096
    F = np.concatenate([rng.uniform(0, 2 * math.pi, (n, N_PMUT)), rng.uniform(1.5, 3, (n, 1)),
                        rng.uniform(0.5, 1, (n, 1))], 1).astype(np.float32)
    U = torch.as_tensor(F, device="cuda")
    T = torch.as_tensor(rng.standard_normal((n, N_OUT), dtype=np.float32) * 0.3, device="cuda")
    y = torch.empty((batch_infer, N_OUT), device="cuda")
    for _ in range(3):
        m.forward(U[:batch_infer], y=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_infer):
        m.forward(U[:batch_infer], y=y)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / n_infer
    idx = torch.as_tensor(np.arange(batch_train, dtype=np.int32), device="cuda")
    for _ in range(3):
        m.train_step(U, T, idx, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_train):
        m.train_step(U, T, idx, 1e-4)
    torch.cuda.synchronize()
    t_tr = (time.perf_counter() - t0) / n_train
    flop = 2.0 * sum(a * b for a, b in zip(widths[:-1], widths[1:]))
    return {"widths": widths, "infer_ms": t_inf * 1e3, "infer_batch": batch_infer,
            "infer_TFLOPs": flop * batch_infer / t_inf / 1e12, "train_step_ms": t_tr * 1e3,
            "train_batch": batch_train, "train_TFLOPs": 3 * flop * batch_train / t_tr / 1e12}


if __name__ == "__main__":
    import json
    print(json.dumps(bench_network()), flush=True)
