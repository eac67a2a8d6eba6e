"""Throughput benchmark: trajectory gate-steps/s of the MPS trajectory simulator with
locally entanglement-optimal unravelling, with the observable error of both precisions.

Workload: 100-qubit open chain, brickwork depth 40 of Haar-random two-qubit gates,
depolarizing p = 0.02 on both qubits after every gate, optimal unravelling of every noise
event, bond dimension chi = 128, 2048 trajectories (synthetic, seeded).  One "step" is one
brickwork layer applied to all trajectories (gate, two noise events, truncation and centre
move for every pair).  Bond capacities are fixed from the first layer on, so the dense kernels
do the work of the saturated bond dimension in every layer.

Passes (each over layers 0 .. K-1, K = 40 by default: the whole circuit, timed from the first
layer through the measurement sweep that gives every trajectory's <Z_i>, <Z_i Z_i+1>; the
discarded weights of every layer feed the certified error estimate inside the timed region;
graphs on, no profiling; W warm-up layers run first on a 64-trajectory batch):
  1. FP32-bulk (c64 contractions; FP64 eigen-solves, unravelling, probabilities,
     observables), its own decisions: `value`;
  2. FP64, recording every event's mixing and branch: `fp64.value`;
  3. FP32-bulk following the FP64 decisions (untimed; layers 8 and 9, saturated, profiled
     per kernel class): the paired per-trajectory observable differences against pass 2
     (the 1e-4 target), `kernels_ms` and the roofline of the dominant kernel;
  4. the oracle replaying trajectory 0 (and 1, if time allows) of pass 2 on the host through
     all K layers: `cpu_baseline` (its rate over layers 8 and 9) and `oracle_error`
     (per-trajectory observable error of passes 2 and 3).
A batch that does not fit in device memory (FP64 at chi = 256) runs in memory waves of
consecutive trajectories with the trajectory offset.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--chi 128] [--traj 2048]
       python bench.py --mixed [--traj 16384] [--steps K] [--warmup W]   (mixed-batch workload)
       python bench.py --cost [--steps K]        (unravelling cost + adjoint, 65536 states)
       python bench.py --lindblad                (Trotterised Lindbladian workloads)
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PROF_NAMES = ["theta", "events", "kraus_pair", "gram", "tridiag", "tri_eig", "hop_eig", "backtransform",
              "recompose", "hop", "idle", "expect", "tridiag_s", "tridiag_l", "backtransform_l"]
# kernel instance timed by each single-instance class
KERNEL = {"theta": "k_theta<float> / k_theta_l (autotuned per shape)", "tridiag": "k_tridiag<256, 6, 2, 512, 4, true>",
          "tridiag_s": "k_tridiag<128, 8, 2, 512, 4, false>",
          "tridiag_l": "k_tridiag<512, 4, 2, 512, 1, true>", "backtransform": "k_bt_tfac + k_bt_panel<256, 512>",
          "backtransform_l": "k_bt_tfac + k_bt_panel<512, 512>", "tri_eig": "k_tri_eig"}
TRIDIAG = {"tridiag_s": (0, 128), "tridiag": (129, 256), "tridiag_l": (257, 512)}
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12}
EIG_SRC = os.path.join(ROOT, "paper_2508_05745_amd", "csrc", "eig.hip")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.txt")
EPS_MAX, DELTA = 4.0, 0.05     # cap of the per-trajectory error bound, failure probability


def caps(n, chi):
    return [min(chi, 2 ** (k + 1), 2 ** (n - k - 1)) for k in range(n - 1)]


def tridiag_bytes(m):
    """HBM bytes the one-stage Householder reduction of an m x m c128 Hermitian matrix must
    read: the lower triangle of the trailing matrix once per column (the matrix-vector
    product), sum over the m - 2 reflectors of r (r + 1) / 2 elements of 16 bytes, r = m - j - 1."""
    return 16.0 * sum(r * (r + 1) // 2 for r in range(2, m))


def algorithmic_work(n, chi, layers, n_traj):
    """Algorithmic work of the timed launches, per kernel class: flops for the contractions
    (theta 32*cl*cm*cr, Gram 32*cl^2*cr (the Hermitian half), recomposition 32 D cl cr),
    back-transformation 8 m^2 D, and for the tridiagonalisations both the flops (16/3 m^3)
    and the HBM bytes of `tridiag_bytes` (m = Gram dimension)."""
    cp = caps(n, chi)
    dl = lambda k: 1 if k == 0 else cp[k - 1]
    dr = lambda k: 1 if k == n - 1 else cp[k]
    w = {k: 0.0 for k in PROF_NAMES}
    by = {k: 0.0 for k in PROF_NAMES}
    for l in layers:
        par = l % 2
        pairs = list(range(par, n - 1, 2))
        for q in pairs:
            cl, cm, cr = dl(q), dr(q), dr(q + 1)
            D = cm
            w["theta"] += 32.0 * cl * cm * cr
            m = 2 * cl if par == 0 else 2 * cr
            w["gram"] += 16.0 * m * cl * cr
            cls = next(k for k, (lo, hi) in TRIDIAG.items() if lo <= m <= hi)
            w[cls] += 16.0 / 3.0 * m ** 3
            by[cls] += tridiag_bytes(m)
            w["backtransform" if m <= 256 else "backtransform_l"] += 8.0 * m * m * D
            w["recompose"] += 32.0 * D * cl * cr
    return {k: v * n_traj for k, v in w.items()}, {k: v * n_traj for k, v in by.items()}


def measured_traffic(kernel, n_traj, chi):
    """HBM bytes per launch of `kernel` from the committed PMC summary (FETCH_SIZE and
    WRITE_SIZE per dispatch, scaled by the same counters on a plain copy kernel), or None when
    the summary is for another workload or the eigensolver source changed since."""
    import hashlib
    if not os.path.exists(TRAFFIC):
        return None
    sha = hashlib.sha256(open(EIG_SRC, "rb").read()).hexdigest()
    for line in open(TRAFFIC):
        if line.startswith("#") or "=" not in line:
            continue
        f = dict(kv.split("=", 1) for kv in line.strip().split(";"))
        if (f.get("kernel") == kernel and f.get("eig_hip_sha256") == sha and int(f["n_traj"]) == n_traj
                and int(f["chi"]) == chi):
            return (float(f["fetch_kib"]) * float(f["fetch_scale"]) + float(f["write_kib"]) * float(f["write_scale"])) * 1024.0
    return None


def n_waves(n_traj, n, chi, prec):
    """Memory waves: the batch runs as 2^k consecutive trajectory ranges (each its own batch,
    draws keyed by the global trajectory index through the trajectory offset) when its state
    and work buffers do not fit in the free device memory."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    free, _ = torch.cuda.mem_get_info()
    waves = 1
    while waves < n_traj:
        sb, wb = M.plan(n_traj // waves, n, chi, prec)
        if sb + wb < 0.9 * free - (2 << 30):
            break
        waves *= 2
    return waves


def warm_up(wl, precision, layers):
    """Untimed: `layers` layers on a small batch of the same shapes (loads the code objects
    and runs each kernel once)."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    if layers <= 0:
        return
    b = M.Batch(64, wl.circuit.n, wl.chi, precision, wl.seed)
    b.set_circuit(wl.circuit, M.OPTIMAL)
    for l in range(min(layers, wl.circuit.depth)):
        b.apply_layer(l)
    b.expect()
    b.sync()
    b.close()
    torch.cuda.synchronize()


def run_pass(wl, precision, L, record=None, replay=None, prof_layers=()):
    """Layers 0 .. L-1 of the workload on all trajectories (in memory waves if needed) and
    the measurement sweep, timed per wave from the first layer through `expect` (per-trajectory
    observables) between device synchronisations, with the discarded weights of every layer
    accumulated into the certified error estimate inside the timed region.  record = (w[l],
    branch[l]) per-layer device tensors over the whole batch that receive the mixings and
    branches; replay = the same structure to follow (paired run).  prof_layers: layers timed
    per kernel class with HIP events (this disables graph replay for them, so a profiled pass
    is not a timed one)."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    c = wl.circuit
    T = wl.n_traj
    waves = n_waves(T, c.n, wl.chi, precision)
    Tw = T // waves
    lib = M.lib()
    lib.mps_profile.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.mps_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    obs = torch.empty((T, 2 * c.n - 1), dtype=torch.float64, device="cuda")
    eb = {k: M.ErrorBound(T, k) for k in (M.STEP_EXACT, M.STEP_PAPER)}
    prof = {k: [0.0, 0] for k in PROF_NAMES}
    dt = 0.0
    for w in range(waves):
        a, z = w * Tw, (w + 1) * Tw
        b = M.Batch(Tw, c.n, wl.chi, precision, wl.seed, traj_offset=a)
        b.set_circuit(c, M.OPTIMAL)
        ebw = {}
        for k, e in eb.items():
            ebw[k] = M.ErrorBound(Tw, k)
            ebw[k].eps_tot = e.eps_tot[a:z]
        d = torch.zeros((Tw, c.n // 2), dtype=torch.float64, device="cuda")
        b.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for l in range(L):
            if prof_layers and l == prof_layers[0]:
                lib.mps_profile(b.h, 1)
            kw = dict(discarded=d)
            if record is not None:
                kw.update(w_record=record[0][l][a:z], branch=record[1][l][a:z])
            if replay is not None:
                kw.update(w_in=replay[0][l][a:z], branch_in=replay[1][l][a:z])
            b.apply_layer(l, **kw)
            for e in ebw.values():
                e.add_layer(d)
            if prof_layers and l == prof_layers[-1]:
                ms = (ctypes.c_double * 32)()
                cnt = (ctypes.c_longlong * 32)()
                nc = lib.mps_profile_read(b.h, ms, cnt, 32)
                for i in range(min(nc, len(PROF_NAMES))):
                    prof[PROF_NAMES[i]][0] += ms[i]
                    prof[PROF_NAMES[i]][1] += cnt[i]
                lib.mps_profile(b.h, 0)
            if l % 8 == 7:
                print(f"#   wave {w + 1}/{waves}: layer {l} queued", file=sys.stderr, flush=True)
        _, _, pt = b.expect()
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
        b.sync()
        obs[a:z] = pt
        b.close()
        del b, d, pt
        torch.cuda.empty_cache()
    est = {}
    for k, e in eb.items():
        name = "exact_step" if k == M.STEP_EXACT else "paper_step"
        est[name] = e.estimate(eps_max=EPS_MAX, delta=DELTA)
        # without the cap: the mean cumulated error itself (no certificate attached)
        est[name + "_uncapped_mean"] = e.estimate(eps_max=1e300, delta=DELTA)[0]
    return dict(seconds=dt, obs=obs.cpu().numpy(), waves=waves, error=est,
                prof={k: tuple(v) for k, v in prof.items()} if prof_layers else None)


def paired_stats(x, y):
    """Per-trajectory differences d = x - y of two runs over the same trajectories: the
    distribution of max_i |d_t,i|, the per-observable mean difference with its standard error
    (the paired comparison of the two runs' estimators), and Hotelling's T^2 test of a zero
    mean difference over all observables jointly (F distribution; correlated observables)."""
    from scipy import stats
    d = x - y
    T, p = d.shape
    per = np.abs(d).max(axis=1)
    md = d.mean(0)
    se = d.std(0, ddof=1) / np.sqrt(T) + 1e-300
    i = int(np.argmax(np.abs(md)))
    out = dict(per_traj_max_abs=dict(max=float(per.max()), median=float(np.median(per)),
                                     p99=float(np.quantile(per, 0.99))),
               mean_diff_max_abs=float(np.abs(md).max()), mean_diff_se_at_max=float(se[i]),
               z_max=float(np.abs(md / se).max()))
    if per.max() > 0 and T > p + 1:
        S = np.cov(d, rowvar=False)
        sol, *_ = np.linalg.lstsq(S, md, rcond=1e-12)
        t2 = float(T * md @ sol)
        rank = int(np.linalg.matrix_rank(S, tol=1e-12 * np.abs(S).max()))
        f = (T - rank) / (rank * (T - 1)) * t2
        out.update(hotelling_t2=t2, hotelling_rank=rank, hotelling_p=float(stats.f.sf(f, rank, T - rank)))
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, L, rec, obs64, obs32p, rate_layers, budget_s=90.0):
    """The oracle MPS (NumPy/LAPACK, FP64) replaying sampled trajectories of the FP64 run
    (its recorded mixings, each checked for completeness and optimality, and its own draws,
    which must reproduce the recorded branches) through all L layers: its rate is taken over
    `rate_layers` (saturated bonds), and its final observables give the per-trajectory error
    of the FP64 run and of the FP32-bulk run that followed the same decisions.  A second
    trajectory is replayed if the first took under a third of the budget."""
    from oracle import mps as omps
    from oracle import sv as osv
    c = wl.circuit
    t_start = time.perf_counter()
    steps, secs, errs = 0, 0.0, []
    for t in (0, 1):
        if t > 0 and time.perf_counter() - t_start > budget_s / 3:
            break
        ws, js = [], []
        for l in range(L):
            wl_ = rec[0][l][t].cpu().numpy()
            bl_ = rec[1][l][t].cpu().numpy()
            for kind, q in osv.sweep_ops(c, l):
                for x in osv.event_qubits(c, l, kind, q):
                    ws.append(wl_[x].T.copy())
                    js.append(int(bl_[x]))
        rp = osv.Replay(ws)
        got = []
        m = omps.MPS(c.n)
        for l in range(L):
            t0 = time.perf_counter()
            omps.trajectory(c, wl.chi, t, wl.seed, mode=3, layer_range=[l], m=m, replay=rp, record=got)
            if l in rate_layers:
                secs += time.perf_counter() - t0
                steps += len(c.pairs(l))
        zi, zz = omps.z_expectations(m)
        ref = np.concatenate([zi, zz])
        errs.append(dict(traj=t, fp64_max_abs=float(np.abs(obs64[t] - ref).max()),
                         fp32_bulk_paired_max_abs=float(np.abs(obs32p[t] - ref).max()),
                         branches_match=js == [r["j"] for r in got],
                         replay_max_eof_gap=float(rp.max_gap)))
        print(f"#   oracle trajectory {t}: {time.perf_counter() - t_start:.1f} s", file=sys.stderr, flush=True)
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    base = dict(value=steps / secs, unit="trajectory gate-steps/s", cores=int(cores), kind="oracle",
                cpu=cpu_model(),
                sample=f"{len(errs)} trajectories of the FP64 run replayed by the oracle (NumPy/LAPACK "
                       f"complex128) through layers 0..{L - 1}; rate over layers {rate_layers[0]}..{rate_layers[-1]}")
    return base, errs


def calibrate_copy(nbytes=1 << 30, reps=4):
    """A plain copy kernel of known size: under `rocprofv3 --pmc FETCH_SIZE` (or WRITE_SIZE)
    each dispatch should read (write) nbytes; the ratio counter / nbytes scales the counters
    taken on the path's kernels."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)   # one elementwise kernel: reads and writes nbytes
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes, "dispatches": reps}))


def bench_mixed(args):
    """Mixed batch: 16384 trajectories, each its own circuit (width 24..64, depth 16..32, chi
    in {16, 32, 64, 128}, depolarizing 0.005..0.03, gates from a 2^16 pool), FP32-bulk, all
    sub-batches of a layer in one graph launch.  Counts the real gates (not the identity
    padding past a trajectory's depth) of the timed layers."""
    import torch

    from paper_2508_05745_amd import inputs as I
    from paper_2508_05745_amd import mpsb as M
    n_traj = args.traj if args.traj != 2048 else 16384
    wl = I.config_mixed(n_traj)
    mc = wl.circuit
    W = args.warmup
    # default: every layer after the warm-up ones (the deepest trajectory's depth)
    K = mc.depth - W if args.steps == 40 else min(args.steps, mc.depth - W)
    b = M.Batch(mc.n_traj, mc.widths, mc.chis, M.FP32_BULK, wl.seed)
    b.set_circuit(mc, M.OPTIMAL)
    for l in range(W):
        b.apply_layer(l)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for l in range(W, W + K):
        b.apply_layer(l)
        # a layer of the whole batch takes seconds: waiting for it costs the next layer's
        # launch latency only, and lets the run report its progress
        torch.cuda.synchronize()
        print(f"#   layer {l}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    b.sync()
    gates = int((mc.gate_id[:, W:W + K, :] >= 0).sum())
    per_chi = {int(c): int((mc.gate_id[mc.chis == c][:, W:W + K, :] >= 0).sum()) for c in np.unique(mc.chis)}
    n_sub = int(np.count_nonzero(np.diff(mc.widths) != 0) + np.count_nonzero(np.diff(mc.chis) != 0) + 1)
    b.close()
    cpu, oracle_err, sched = None, None, None
    if not args.no_cpu:
        cpu, oracle_err, sched = mixed_oracle_check(wl)
    line = {
        "metric": "trajectory gate-steps/s (mixed batch)", "value": gates / dt, "unit": "trajectory gate-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": 1e3 * dt / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64 contractions (fp32) + fp64 eig/unravel",
        "data": "synthetic (seeded per-trajectory Haar brickwork from a 2^16-gate pool)",
        "config": {"workload": wl.name, "n_traj": mc.n_traj, "max_width": mc.n, "max_depth": mc.depth,
                   "sub_batches_upper_bound": n_sub, "timed_layers": [W, W + K - 1],
                   "gate_steps_timed": gates, "gate_steps_per_chi": per_chi},
        "oracle_error": oracle_err, "cpu_baseline": cpu, "schedule": sched,
    }
    print(json.dumps(line))


def mixed_oracle_check(wl):
    """Untimed second pass of the whole mixed batch (same seeds, recording every mixing and
    branch), then the oracle MPS replays one trajectory of each chi class (the middle one of
    the class, sorted by width) from layer 0: its branches must match, its mixings are checked
    for completeness and optimality, and its final observables give the trajectory's error."""
    import torch

    from oracle import mps as omps
    from oracle import sv as osv
    from paper_2508_05745_amd import mpsb as M
    mc = wl.circuit
    sample = []
    for chi in np.unique(mc.chis):
        idx = np.flatnonzero(mc.chis == chi)
        sample.append(int(idx[len(idx) // 2]))
    st = torch.as_tensor(sample).cuda()
    b = M.Batch(mc.n_traj, mc.widths, mc.chis, M.FP32_BULK, wl.seed)
    b.set_circuit(mc, M.OPTIMAL)
    T, W = mc.n_traj, mc.n
    w = torch.zeros((T, W, 4, 4), dtype=torch.complex128, device="cuda")
    br = torch.zeros((T, W), dtype=torch.int32, device="cuda")
    ws, brs = [], []
    sched = None
    for l in range(mc.depth):
        if l == SCHED_LAYERS[0]:
            b.profile(2)
        b.apply_layer(l, branch=br, w_record=w)
        if l == SCHED_LAYERS[1]:
            sched = schedule_report(mc, *b.schedule_read())
            b.profile(0)
        ws.append(w[st].cpu().numpy())
        brs.append(br[st].cpu().numpy())
        if l % 4 == 3:
            print(f"#   recorded pass: layer {l}", file=sys.stderr, flush=True)
    _, _, pt = b.expect()
    pt = pt[st].cpu().numpy()
    b.sync()
    b.close()
    del w, br
    errs, steps, secs = [], 0, 0.0
    for i, t in enumerate(sample):
        c = mc.trajectory_circuit(t)
        wl_, js = [], []
        for l in range(c.depth):
            for kind, q in osv.sweep_ops(c, l):
                for x in osv.event_qubits(c, l, kind, q):
                    wl_.append(ws[l][i, x].T.copy())
                    js.append(int(brs[l][i, x]))
        rp = osv.Replay(wl_)
        got = []
        t0 = time.perf_counter()
        m, _ = omps.trajectory(c, int(mc.chis[t]), t, wl.seed, mode=3, record=got, replay=rp)
        secs += time.perf_counter() - t0
        steps += sum(len(c.pairs(l)) for l in range(c.depth))
        zi, zz = omps.z_expectations(m)
        ref = np.concatenate([zi, zz])
        nobs = 2 * c.n - 1
        errs.append(dict(traj=t, width=int(c.n), depth=int(c.depth), chi=int(mc.chis[t]),
                         fp32_bulk_max_abs=float(np.abs(pt[i][:nobs] - ref).max()),
                         branches_match=js == [r["j"] for r in got], replay_max_eof_gap=float(rp.max_gap),
                         replay_max_incomplete=float(rp.max_incomplete)))
        print(f"#   oracle trajectory {t} (chi {mc.chis[t]}, width {c.n}): {secs:.1f} s, "
              f"max |d<O>| {errs[-1]['fp32_bulk_max_abs']:.1e}", file=sys.stderr, flush=True)
    base = dict(value=steps / secs, unit="trajectory gate-steps/s", cores=_cores(), kind="oracle", cpu=cpu_model(),
                sample=f"{len(sample)} trajectories (one per chi class) of an untimed recorded FP32-bulk pass "
                       f"replayed by the oracle (NumPy/LAPACK complex128) through all their layers")
    return base, errs, sched


# layers of the mixed batch's recorded pass whose member schedule is timed (every member has
# work in them: depths start at 16)
SCHED_LAYERS = (8, 11)


def schedule_report(mc, first, count, stream, busy, elapsed, layers):
    """Per-chi-class rates and stream utilisation from the member schedule of timed layers.
    A member's gate-steps are the real gates (not the identity padding past a trajectory's own
    depth) of its trajectories in those layers.  The rate of a chi class is its trajectory
    gate-steps over its members' summed busy time (the rate of the class on the stream slots it
    occupied); utilisation = summed busy time / (streams x elapsed)."""
    lo, hi = SCHED_LAYERS
    ns = min(4, len(first))
    per = {}
    total = 0
    for f, c, ms in zip(first, count, busy):
        chi = int(mc.chis[f])
        g = int((mc.gate_id[f:f + c, lo:hi + 1, :] >= 0).sum())
        d = per.setdefault(chi, [0, 0.0, 0])
        d[0] += g
        d[1] += ms
        d[2] += 1
        total += g
    return {
        "layers": [lo, hi], "layers_timed": int(layers), "members": int(len(first)), "streams": ns,
        "assignment": "round-robin over the members sorted by (chi, width)",
        "elapsed_ms": elapsed, "busy_ms": float(np.sum(busy)),
        "utilisation_busy_over_streams_x_elapsed": float(np.sum(busy) / (ns * elapsed)) if elapsed > 0 else None,
        "rate_all": total / (elapsed * 1e-3) if elapsed > 0 else None,
        "per_chi": {str(k): {"gate_steps": v[0], "busy_ms": v[1], "members": v[2],
                             "rate_on_its_streams": v[0] / (v[1] * 1e-3) if v[1] > 0 else None}
                    for k, v in sorted(per.items())},
        "note": "direct launches with an event pair around every member's layer (no layer graphs)",
    }


def bench_cost(args):
    """Unravelling cost and adjoint on 65536 independent two-site states (chi 64 on each side,
    complex Gaussian, normalised, c64, drawn on the device), 4-Kraus depolarizing p = 0.02,
    mixing parameters N(0, 0.1^2) around Haar reference unitaries: one step = the linear
    cost of every state and its adjoint gradient.  Between the noisy qubit and the rest of the
    block (default) the forward is the reduction of the reduced qubit state, HBM-bound (16 chi^2
    bytes read per state); across the block's internal bond (--bond) it is the block Gram
    matrix, matrix-core bound (4 (2 chi)^3 FP64 flops of a Hermitian product per state)."""
    import torch

    from paper_2508_05745_amd import inputs as I
    from paper_2508_05745_amd import mpsb as M
    bond = bool(getattr(args, "bond", False))
    B, chi = (16384, 64) if bond else (65536, 64)
    th = I.random_two_site_states_torch(B, chi, chi, seed=4004)
    pp = torch.as_tensor(I.random_mixing_params(B, seed=4005)).cuda()
    uu = torch.as_tensor(I.haar_unitaries(B, seed=4006)).cuda()
    k = I.depolarizing(0.02)

    def fwd_bwd():
        if bond:
            f, rho, nm, k4 = M.unravel_cost_bond(th, k, pp, uu, 0)
            return lambda: M.unravel_cost_bond_grad(rho, nm, k4, pp, uu, 0, None)
        f, rho, k4 = M.unravel_cost(th, k, pp, uu, 0)
        return lambda: M.unravel_cost_grad(rho, k4, pp, uu, 0, None)

    W, K = max(args.warmup, 1), args.steps
    for _ in range(W):
        fwd_bwd()()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record()
        bwd_call = fwd_bwd()
        e1.record()
        bwd_call()
        e2.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fwd = sum(a.elapsed_time(b) for a, b, _ in ev) / K
    bwd = sum(b.elapsed_time(c) for _, b, c in ev) / K
    cpu = None
    if not args.no_cpu:
        from oracle import cost as CO
        sample = np.linspace(0, B - 1, 4096).astype(np.int64)
        ths = th[torch.as_tensor(sample).cuda()].cpu().numpy().astype(np.complex128)
        params, uref = pp.cpu().numpy(), uu.cpu().numpy()
        t1, n = time.perf_counter(), 0
        while n < len(sample) and (time.perf_counter() - t1 < 15.0 or n == 0):
            if bond:
                CO.bond_grad_torch(ths[n], k, params[sample[n]], uref[sample[n]], 0)
            else:
                r = CO.rho_from_theta(ths[n])
                CO.grad_torch(r / np.trace(r).real, k, params[sample[n]], uref[sample[n]], 0)
            n += 1
        how = "branch Gram matrices + torch-CPU complex128 autograd" if bond else "NumPy reduction + torch-CPU complex128 autograd"
        cpu = dict(value=n / (time.perf_counter() - t1), unit="states/s", cores=_cores(), kind="oracle", cpu=cpu_model(),
                   sample=f"{n} states of the batch ({how})")
    if bond:
        flops = B * 4.0 * (2 * chi) ** 3
        roof = dict(bound="mfma", kernel="k_bond_moments<float> + k_cost_eval (forward)",
                    achieved=flops / (fwd * 1e-3) / 1e12, peak=PEAK["fp64"] / 1e12, unit="TFLOP/s",
                    frac=flops / (fwd * 1e-3) / PEAK["fp64"], traffic=None, flops_per_launch=flops, avg_launch_ms=fwd)
        metric, wl = "two-site states/s (internal-bond unravelling cost + adjoint)", f"bondcost-{B}states-chi{chi}-dep0.02"
        dtype = "c64 states, fp64 Gram (matrix cores) / cost / adjoint"
    else:
        nbytes = B * chi * 4 * chi * 8.0
        roof = dict(bound="hbm", kernel="k_cost_rho<float> + k_cost_eval (forward)", achieved=nbytes / (fwd * 1e-3) / 1e9,
                    peak=PEAK["hbm"] / 1e9, unit="GB/s", frac=nbytes / (fwd * 1e-3) / PEAK["hbm"], traffic=None,
                    bytes_per_launch=nbytes, avg_launch_ms=fwd)
        metric, wl = "two-site states/s (unravelling cost + adjoint)", f"cost-{B}states-chi{chi}-dep0.02"
        dtype = "c64 states, fp64 reduction / cost / adjoint"
    line = {
        "metric": metric, "value": B * K / dt, "unit": "states/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": 1e3 * dt / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic (seeded complex-Gaussian states, depolarizing p=0.02)",
        "config": {"workload": wl, "n_states": B, "chi": chi},
        "roofline": roof, "backward_ms": bwd, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def bench_lindblad(args):
    """Trotterised Lindbladian workloads of the paper's two studies: the fixed Heisenberg-type
    Hamiltonian with amplitude damping (16 qubits, chi 50, 500 trajectories, 600 layers of
    dt = 0.01 / 2, amplitude damping 0.002 per layer) and a random translation-invariant one
    (12 qubits, chi 20, 1000 trajectories, 600 layers); optimal unravelling, FP32-bulk, timed
    from the first layer through the measurement sweep."""
    import torch

    from paper_2508_05745_amd import inputs as I
    from paper_2508_05745_amd import mpsb as M
    runs = []
    for m, chi, T in ((I.lindblad_heisenberg(n=16, steps=300, dt=0.01, gamma_ad=0.002), 50, 500),
                      (I.lindblad_random_ti(n=12, steps=300, dt=0.01, gamma_ad=0.002, seed=1), 20, 1000)):
        c = M.lindblad_circuit(m)
        L = min(args.steps, c.depth) if args.steps != 40 else c.depth
        b = M.Batch(T, c.n, chi, M.FP32_BULK, 2007)
        b.set_circuit(c, M.OPTIMAL)
        b.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for l in range(L):
            b.apply_layer(l)
        b.expect()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.sync()
        b.close()
        gates = T * sum(len(c.pairs(l)) for l in range(L))
        runs.append(dict(workload=f"{m.name}-chi{chi}-{T}traj", layers=L, value=gates / dt, seconds=dt))
        print(f"# {runs[-1]['workload']}: {dt:.2f} s, {gates / dt:.0f} gate-steps/s", file=sys.stderr, flush=True)
    line = {
        "metric": "trajectory gate-steps/s (Lindbladian workloads)", "value": runs[0]["value"],
        "unit": "trajectory gate-steps/s", "n_gpus": 1, "steps": runs[0]["layers"], "warmup": 0,
        "ms_per_step": 1e3 * runs[0]["seconds"] / runs[0]["layers"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 contractions (fp32) + fp64 eig/unravel",
        "data": "synthetic (the paper's Heisenberg-type and seeded random translation-invariant Lindbladians)",
        "config": {"workload": runs[0]["workload"], "runs": runs},
    }
    print(json.dumps(line))


def _cores():
    try:
        from threadpoolctl import threadpool_info
        return int(max([d.get("num_threads", 1) for d in threadpool_info()] + [1]))
    except Exception:
        return os.cpu_count() or 1


def roofline(work, nbytes, prof, wl):
    """Roofline of the dominant kernel class (largest HIP-event time in the profiled pass;
    each class times one kernel instance).  The eigensolver's tridiagonalisation is bounded
    by the FP64 units (16/3 m^3 flops per m x m matrix, on the VALU); its one-stage HBM byte
    model and the counted traffic are reported beside it."""
    dom = max(prof, key=lambda k: prof[k][0])
    ms, cnt = prof[dom]
    sec = ms * 1e-3
    rate = work.get(dom, 0.0) / sec if sec > 0 else 0.0
    if dom in TRIDIAG:
        roof = dict(bound="alu", achieved=rate / 1e12, peak=PEAK["fp64"] / 1e12, unit="TFLOP/s",
                    frac=rate / PEAK["fp64"], traffic=measured_traffic(KERNEL[dom], wl.n_traj, wl.chi),
                    hbm_model=dict(bytes_per_launch=nbytes[dom] / max(cnt, 1),
                                   achieved_gbs=nbytes[dom] / sec / 1e9 if sec > 0 else 0.0,
                                   frac_of_8tbs=nbytes[dom] / sec / PEAK["hbm"] if sec > 0 else 0.0))
    elif dom in ("theta", "gram", "recompose"):
        roof = dict(bound="mfma", achieved=rate / 1e12, peak=PEAK["fp32"] / 1e12, unit="TFLOP/s",
                    frac=rate / PEAK["fp32"], traffic=None)
    else:
        roof = dict(bound="alu", achieved=rate / 1e12, peak=PEAK["fp64"] / 1e12, unit="TFLOP/s",
                    frac=rate / PEAK["fp64"], traffic=None)
    roof.update(kernel=KERNEL.get(dom, dom), launches=int(cnt), avg_launch_ms=ms / max(cnt, 1),
                flops_per_launch=work.get(dom, 0.0) / max(cnt, 1))
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40, help="layers timed from layer 0 (40 = the whole circuit)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed layers on a 64-trajectory batch first")
    ap.add_argument("--chi", type=int, default=128)
    ap.add_argument("--traj", type=int, default=2048)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mixed", action="store_true", help="the mixed-batch workload instead of the headline one")
    ap.add_argument("--cost", action="store_true", help="the unravelling cost / adjoint workload (65536 states)")
    ap.add_argument("--bond", action="store_true",
                    help="with --cost: the cost across the block's internal bond (16384 states)")
    ap.add_argument("--lindblad", action="store_true", help="the Trotterised Lindbladian workloads")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB elementwise copy kernel 4 times (HBM counter scale)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; a run on several GPUs would give each GPU a "
                                   "disjoint trajectory range (designed, not built)", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.mixed:
        bench_mixed(args)
        return
    if args.cost:
        bench_cost(args)
        return
    if args.lindblad:
        bench_lindblad(args)
        return
    import torch

    from paper_2508_05745_amd import inputs as I
    from paper_2508_05745_amd import mpsb as M
    wl = I.config_wide(chi=args.chi, n_traj=args.traj)
    c = wl.circuit
    W, K = args.warmup, args.steps
    T = wl.n_traj
    if not 2 <= K <= c.depth:
        raise SystemExit(f"--steps must lie in 2..{c.depth}")
    # kernel classes and the oracle's rate are taken on two saturated layers
    prof_layers = [8, 9] if K >= 10 else [K - 2, K - 1]
    gate_steps = T * sum(len(c.pairs(l)) for l in range(K))
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)
    log(f"warm-up: {W} layers on 64 trajectories")
    warm_up(wl, M.FP32_BULK, W)
    log(f"fp32-bulk: layers 0..{K - 1} and the measurement sweep, {gate_steps} gate-steps")
    p32 = run_pass(wl, M.FP32_BULK, K)
    value = gate_steps / p32["seconds"]
    log(f"fp32-bulk: {p32['seconds']:.3f} s -> {value:.1f} gate-steps/s")
    fp64, paired, rec = None, None, None
    if not args.no_fp64:
        warm_up(wl, M.FP64, W)
        rec = ([torch.zeros((T, c.n, 4, 4), dtype=torch.complex128, device="cuda") for _ in range(K)],
               [torch.zeros((T, c.n), dtype=torch.int32, device="cuda") for _ in range(K)])
        log("fp64 (recording every decision)")
        p64 = run_pass(wl, M.FP64, K, record=rec)
        log(f"fp64: {p64['seconds']:.3f} s -> {gate_steps / p64['seconds']:.1f} gate-steps/s")
        log(f"fp32-bulk following the fp64 decisions (paired; layers {prof_layers} profiled)")
        pp = run_pass(wl, M.FP32_BULK, K, replay=rec, prof_layers=prof_layers)
        fp64 = dict(value=gate_steps / p64["seconds"], ms_per_step=1e3 * p64["seconds"] / K, waves=p64["waves"],
                    certified_error=p64["error"],
                    vs_fp32_bulk_own_decisions=paired_stats(p32["obs"], p64["obs"]))
        paired = paired_stats(pp["obs"], p64["obs"])
        paired["target"] = 1e-4
        log(f"paired fp32-bulk vs fp64: max |d<O>| {paired['per_traj_max_abs']['max']:.2e}, "
            f"max |mean d| {paired['mean_diff_max_abs']:.2e}")
    else:
        log(f"fp32-bulk pass, layers {prof_layers} profiled")
        pp = run_pass(wl, M.FP32_BULK, K, prof_layers=prof_layers)
    prof = pp["prof"]
    work, nbytes = algorithmic_work(c.n, wl.chi, prof_layers, T)
    roof = roofline(work, nbytes, prof, wl)
    kern = {k: dict(ms=v[0], launches=int(v[1])) for k, v in prof.items() if v[1] > 0}
    th = prof.get("theta", (0, 1))
    theta_rate = work["theta"] / (th[0] * 1e-3) if th[0] > 0 else 0.0
    cpu, oracle_err = None, None
    if not args.no_cpu and rec is not None:
        log("oracle replay of sampled fp64 trajectories (cpu baseline)")
        cpu, oracle_err = cpu_baseline(wl, K, rec, p64["obs"], pp["obs"], prof_layers)
    line = {
        "metric": "trajectory gate-steps/s at chi=128 (FP32-bulk vs FP64) + <O> error vs oracle",
        "value": value, "unit": "trajectory gate-steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": 1e3 * p32["seconds"] / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 contractions (fp32) + fp64 eig/unravel",
        "data": "synthetic (seeded Haar brickwork, depolarizing p=0.02)",
        "config": {"workload": wl.name, "n_qubits": c.n, "depth": c.depth, "chi": wl.chi,
                   "n_traj": T, "unravel": "optimal",
                   "timed": f"layers 0..{K - 1} + measurement sweep (<Z_i>, <Z_i Z_i+1> per trajectory)",
                   "waves": p32["waves"], "parallelism": "trajectories (1 GPU)"},
        "roofline": roof, "theta_roofline": dict(kernel=KERNEL["theta"], bound="mfma", achieved=theta_rate / 1e12,
                                                 peak=PEAK["fp32"] / 1e12, unit="TFLOP/s",
                                                 frac=theta_rate / PEAK["fp32"]),
        "kernels_ms": kern,
        "kernels_ms_pass": f"fp32-bulk, layers {prof_layers[0]}..{prof_layers[-1]}"
                           + (" following the fp64 decisions" if rec is not None else ""),
        "certified_error": dict(p32["error"], eps_max=EPS_MAX, delta=DELTA,
                                meaning="(eps_hat, Hoeffding buffer, bound): with probability >= 1-delta the "
                                        "trace distance of the sampled mixture to the exact state is <= bound"),
        "fp64": fp64, "paired_fp32_bulk_vs_fp64": paired, "oracle_error": oracle_err, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
