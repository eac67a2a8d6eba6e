"""Throughput benchmark: trajectory gate-steps/s of the MPS trajectory simulator with
locally entanglement-optimal unravelling.

Workload: 100-qubit open chain, brickwork depth 40 of Haar-random two-qubit gates,
depolarizing p = 0.02 on both qubits after every gate, optimal unravelling of every noise
event, bond dimension chi = 128, 2048 trajectories (synthetic, seeded).  One "step" is one
brickwork layer applied to all trajectories (gate, two noise events, truncation and centre
move for every pair).  Bond capacities are fixed from the first layer on, so the dense kernels
do the work of the saturated bond dimension in every layer.

The FP32-bulk path (c64 contractions, FP64 eigen-solves / unravelling / probabilities /
observables) gives `value`; the full-FP64 path is timed on the same steps and the paired
difference of the per-trajectory observables is reported.  The default warm-up of 8 layers
brings the bulk bonds to chi = 128 (a bond can grow by a factor 2 per layer), so the timed
layers 8 and 9 run on saturated spectra as most layers of the 40-layer circuit do.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--chi 128] [--traj 2048]
       python bench.py --mixed [--traj 16384] [--steps K] [--warmup W]   (mixed-batch workload)
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
KERNEL = {"theta": "k_theta<float> / k_theta_l (autotuned per shape)", "tridiag": "k_tridiag<256, 6, 2, 512, 4>", "tridiag_s": "k_tridiag<128, 8, 2, 512, 4>",
          "tridiag_l": "k_tridiag<512, 4, 2, 512, 1>", "backtransform": "k_bt_tfac + k_bt_panel<256, 512>",
          "backtransform_l": "k_bt_tfac + k_bt_panel<512, 512>", "tri_eig": "k_tri_eig"}
TRIDIAG = {"tridiag_s": (0, 128), "tridiag": (129, 256), "tridiag_l": (257, 512)}
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12}
EIG_SRC = os.path.join(ROOT, "paper_2508_05745_amd", "csrc", "eig.hip")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.txt")


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


def run_gpu(workload, layers_warm, layers_timed, precision, profile=True):
    import torch

    from paper_2508_05745_amd import mpsb as M
    c = workload.circuit
    b = M.Batch(workload.n_traj, c.n, workload.chi, precision, workload.seed)
    b.set_circuit(c, M.OPTIMAL)
    for l in layers_warm:
        b.apply_layer(l)
    b.sync()
    lib = M.lib()
    if profile:
        lib.mps_profile.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.mps_profile(b.h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for l in layers_timed:
        b.apply_layer(l)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b.sync()
    prof = None
    if profile:
        ms = (ctypes.c_double * 32)()
        cnt = (ctypes.c_longlong * 32)()
        lib.mps_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        nc = lib.mps_profile_read(b.h, ms, cnt, 32)
        prof = {PROF_NAMES[i]: (ms[i], cnt[i]) for i in range(min(nc, len(PROF_NAMES)))}
        lib.mps_profile(b.h, 0)
    _, _, pt = b.expect()
    b.sync()
    obs = pt.cpu().numpy()
    b.close()
    del b
    torch.cuda.empty_cache()
    return t1 - t0, prof, obs


def cpu_baseline(workload, budget_s=25.0):
    """The oracle MPS (NumPy, FP64) on one trajectory of the same circuit and chi: untimed
    layers until the bond dimension saturates (or half the budget), then timed layers."""
    from oracle import mps as omps
    from oracle import sv as osv
    c = workload.circuit
    m = omps.MPS(c.n)
    t_start = time.perf_counter()
    l = 0
    while l < c.depth and time.perf_counter() - t_start < 0.5 * budget_s:
        omps.trajectory(c, workload.chi, 0, workload.seed, layer_range=[l], m=m)
        l += 1
        if max(m.bond_dims()) >= workload.chi and l >= 14:
            break
    warm = l
    t0 = time.perf_counter()
    steps = 0
    while l < c.depth and (time.perf_counter() - t0 < 0.4 * budget_s or steps == 0):
        omps.trajectory(c, workload.chi, 0, workload.seed, layer_range=[l], m=m)
        steps += len(c.pairs(l))
        l += 1
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return dict(value=steps / dt, unit="trajectory gate-steps/s", cores=int(cores), kind="oracle",
                sample=f"1 trajectory, layers {warm}..{l - 1} (after {warm} untimed layers, max bond "
                       f"{max(m.bond_dims())}) of the same chi={workload.chi} circuit, "
                       f"NumPy/LAPACK complex128")


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
    W, K = args.warmup, args.steps
    b = M.Batch(mc.n_traj, mc.widths, mc.chis, M.FP32_BULK, wl.seed)
    b.set_circuit(mc, M.OPTIMAL)
    for l in range(W):
        b.apply_layer(l)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for l in range(W, W + K):
        b.apply_layer(l)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.sync()
    gates = int((mc.gate_id[:, W:W + K, :] >= 0).sum())
    per_chi = {int(c): int((mc.gate_id[mc.chis == c][:, W:W + K, :] >= 0).sum()) for c in np.unique(mc.chis)}
    n_sub = int(np.count_nonzero(np.diff(mc.widths) != 0) + np.count_nonzero(np.diff(mc.chis) != 0) + 1)
    b.close()
    line = {
        "metric": "trajectory gate-steps/s (mixed batch)", "value": gates / dt, "unit": "trajectory gate-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": 1e3 * dt / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64 contractions (fp32) + fp64 eig/unravel",
        "data": "synthetic (seeded per-trajectory Haar brickwork from a 2^16-gate pool)",
        "config": {"workload": wl.name, "n_traj": mc.n_traj, "max_width": mc.n, "max_depth": mc.depth,
                   "sub_batches_upper_bound": n_sub, "timed_layers": [W, W + K - 1],
                   "gate_steps_timed": gates, "gate_steps_per_chi": per_chi},
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--chi", type=int, default=128)
    ap.add_argument("--traj", type=int, default=2048)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mixed", action="store_true", help="the mixed-batch workload instead of the headline one")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB elementwise copy kernel 4 times (HBM counter scale)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.mixed:
        if args.gpus != 1:
            print(json.dumps({"error": "this library runs on one GPU", "n_gpus": args.gpus}))
            sys.exit(2)
        bench_mixed(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; multi-GPU sharding (disjoint "
                                   "trajectory ranges) is designed but not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    from paper_2508_05745_amd import inputs as I
    from paper_2508_05745_amd import mpsb as M
    wl = I.config_wide(chi=args.chi, n_traj=args.traj)
    c = wl.circuit
    W, K = args.warmup, args.steps
    if W + K > c.depth:
        raise SystemExit("warmup + steps exceeds the circuit depth (40)")
    warm, timed = list(range(W)), list(range(W, W + K))
    gate_steps = wl.n_traj * sum(len(c.pairs(l)) for l in timed)
    print(f"# fp32-bulk: {W} warmup + {K} timed layers, {gate_steps} gate-steps", file=sys.stderr, flush=True)
    dt32, prof, obs32 = run_gpu(wl, warm, timed, M.FP32_BULK)
    value = gate_steps / dt32
    print(f"# fp32-bulk: {dt32:.3f} s -> {value:.1f} gate-steps/s", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        dt64, prof64, obs64 = run_gpu(wl, warm, timed, M.FP64, profile=False)
        # the optimal decomposition is not unique, so paired FP32 / FP64 trajectories can
        # take different (equally optimal) branches: compare the trajectory averages
        nt = obs32.shape[0]
        se = np.sqrt(obs32.var(0, ddof=1) / nt + obs64.var(0, ddof=1) / nt) + 1e-300
        dmean = np.abs(obs32.mean(0) - obs64.mean(0))
        fp64 = dict(value=gate_steps / dt64, ms_per_step=1e3 * dt64 / K,
                    mean_obs_abs_diff_max=float(dmean.max()), mean_obs_z_max=float((dmean / se).max()),
                    observables=f"<Z_i>, <Z_i Z_i+1> after layer {W + K - 1}, {nt} trajectories each")
        print(f"# fp64: {dt64:.3f} s, max |d mean<O>| {dmean.max():.2e} (z {float((dmean / se).max()):.2f})",
              file=sys.stderr, flush=True)
    # roofline of the dominant kernel class (each timed class is one kernel instance)
    work, nbytes = algorithmic_work(c.n, wl.chi, timed, wl.n_traj)
    dom = max(prof, key=lambda k: prof[k][0])
    ms, cnt = prof[dom]
    sec = ms * 1e-3
    if dom in TRIDIAG:
        # one pass over the trailing lower triangle per column: about 2 flop per byte, far
        # below the FP64 ridge point (78.6 TFLOP/s / 8 TB/s), so HBM bounds it
        achieved = nbytes[dom] / sec if sec > 0 else 0.0
        roof = dict(bound="hbm", achieved=achieved / 1e9, peak=PEAK["hbm"] / 1e9, unit="GB/s",
                    frac=achieved / PEAK["hbm"],
                    traffic=measured_traffic(KERNEL[dom], wl.n_traj, wl.chi),
                    algorithmic_bytes_per_launch=nbytes[dom] / max(cnt, 1),
                    fp64_tflops=work[dom] / sec / 1e12 if sec > 0 else 0.0)
    elif dom in ("theta", "gram", "recompose"):
        achieved = work[dom] / sec if sec > 0 else 0.0
        roof = dict(bound="mfma", achieved=achieved / 1e12, peak=PEAK["fp32"] / 1e12, unit="TFLOP/s",
                    frac=achieved / PEAK["fp32"], traffic=None)
    else:
        achieved = work.get(dom, 0.0) / sec if sec > 0 else 0.0
        roof = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK["fp64"] / 1e12, unit="TFLOP/s",
                    frac=achieved / PEAK["fp64"], traffic=None)
    roof.update(kernel=KERNEL.get(dom, dom), launches=int(cnt), avg_launch_ms=ms / max(cnt, 1))
    kern = {k: dict(ms=v[0], launches=int(v[1])) for k, v in prof.items() if v[1] > 0}
    th = prof.get("theta", (0, 1))
    theta_rate = work["theta"] / (th[0] * 1e-3) if th[0] > 0 else 0.0
    cpu = None if args.no_cpu else cpu_baseline(wl)
    line = {
        "metric": "trajectory gate-steps/s at chi=128 (FP32-bulk vs FP64) + <O> error vs oracle",
        "value": value, "unit": "trajectory gate-steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": 1e3 * dt32 / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 contractions (fp32) + fp64 eig/unravel",
        "data": "synthetic (seeded Haar brickwork, depolarizing p=0.02)",
        "config": {"workload": wl.name, "n_qubits": c.n, "depth": c.depth, "chi": wl.chi,
                   "n_traj": wl.n_traj, "unravel": "optimal", "parallelism": "trajectories (1 GPU)"},
        "roofline": roof, "theta_roofline": dict(kernel=KERNEL["theta"], bound="mfma", achieved=theta_rate / 1e12,
                                                 peak=PEAK["fp32"] / 1e12, unit="TFLOP/s",
                                                 frac=theta_rate / PEAK["fp32"]),
        "kernels_ms": kern, "fp64": fp64, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
