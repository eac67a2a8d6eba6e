"""Host logic of bench.py (no GPU): the algorithmic bytes of the tridiagonalisation roofline,
the lookup of the committed HBM-traffic summary (keyed by the eigensolver source), and the
one-GPU guard."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tridiag_bytes_tetrahedral_closed_form():
    # reflector j reads the trailing lower triangle of size r = m - j - 1, j = 0 .. m - 3, i.e.
    # r = 2 .. m - 1; sum_{r=1}^{N} r (r + 1) / 2 is the tetrahedral number N (N + 1) (N + 2) / 6
    for m in (3, 4, 17, 128, 256, 512):
        tet = (m - 1) * m * (m + 1) // 6 - 1
        assert bench.tridiag_bytes(m) == 16.0 * tet
    assert abs(bench.tridiag_bytes(256) - 44.74e6) < 0.01e6


def _line(kernel, n_traj, chi, sha, fetch=100.0, write=50.0, fs=2.0, ws=1.0):
    return (f"kernel={kernel};n_traj={n_traj};chi={chi};dispatches=3;fetch_kib={fetch};write_kib={write};"
            f"fetch_scale={fs};write_scale={ws};eig_hip_sha256={sha}\n")


def test_measured_traffic_is_keyed_by_source_and_workload(tmp_path, monkeypatch):
    sha = hashlib.sha256(open(bench.EIG_SRC, "rb").read()).hexdigest()
    f = tmp_path / "traffic.txt"
    f.write_text("# header\n" + _line("kA", 2048, 128, sha) + _line("kB", 2048, 128, "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC", str(f))
    assert bench.measured_traffic("kA", 2048, 128) == (100.0 * 2.0 + 50.0 * 1.0) * 1024.0
    assert bench.measured_traffic("kB", 2048, 128) is None        # counters of another source
    assert bench.measured_traffic("kA", 1024, 128) is None        # another workload
    assert bench.measured_traffic("kA", 2048, 256) is None
    assert bench.measured_traffic("kC", 2048, 128) is None
    monkeypatch.setattr(bench, "TRAFFIC", str(tmp_path / "absent.txt"))
    assert bench.measured_traffic("kA", 2048, 128) is None


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_paired_stats_detects_a_shift_and_accepts_none():
    import numpy as np
    rng = np.random.default_rng(3)
    T, p = 2048, 40
    mix = rng.standard_normal((p, p)) / np.sqrt(p)          # correlated observables
    y = rng.standard_normal((T, p)) @ mix
    x0 = y + 1e-3 * (rng.standard_normal((T, p)) @ mix)       # same mean
    s0 = bench.paired_stats(x0, y)
    assert s0["hotelling_rank"] == p and s0["hotelling_p"] > 1e-3
    assert abs(s0["per_traj_max_abs"]["max"] - np.abs(x0 - y).max()) == 0.0
    x1 = x0.copy()
    x1[:, 7] += 2e-4                                         # a shift of 6 standard errors in one
    s1 = bench.paired_stats(x1, y)
    assert s1["hotelling_p"] < 1e-4 and s1["z_max"] > 4.0
    same = bench.paired_stats(y, y)
    assert same["per_traj_max_abs"]["max"] == 0.0 and "hotelling_t2" not in same


def test_tridiag_roofline_is_fp64_flops():
    class WL:
        n_traj, chi = 2048, 128
    work, nbytes = bench.algorithmic_work(100, 128, [8, 9], 2048)
    prof = {k: (0.0, 0) for k in bench.PROF_NAMES}
    cp = bench.caps(100, 128)
    launches = sum(1 for l in (8, 9) for q in range(l % 2, 99, 2)
                   if 129 <= (2 * cp[q - 1] if l % 2 == 0 else 2 * cp[q + 1]) <= 256)
    prof["tridiag"] = (2000.0, launches)
    prof["theta"] = (100.0, 99)
    r = bench.roofline(work, nbytes, prof, WL)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    flops = 16.0 / 3.0 * 256 ** 3 * 2048                     # one m = 256 Gram per trajectory per launch
    assert abs(r["flops_per_launch"] - flops) / flops < 0.02
    assert abs(r["frac"] - r["achieved"] / 78.6) < 1e-12


def test_schedule_report_rates_and_utilisation():
    """Two chi classes, three members; gate-steps come from the gate table (identity -1 past a
    trajectory's depth is not counted), rates from the members' busy time, utilisation from
    the summed busy time over streams x elapsed."""
    import numpy as np

    class MC:
        pass

    mc = MC()
    mc.chis = np.array([16, 16, 64, 64, 64])
    lo, hi = bench.SCHED_LAYERS
    L = hi + 2
    mc.gate_id = np.full((5, L, 3), -1)
    mc.gate_id[:, lo:hi + 1, :2] = 7            # two real gates per trajectory and timed layer
    mc.gate_id[4, hi, :] = -1                   # trajectory 4 ends before the last timed layer
    nl = hi - lo + 1
    first, count = np.array([0, 2, 4]), np.array([2, 2, 1])
    busy = np.array([2.0, 6.0, 4.0])
    r = bench.schedule_report(mc, first, count, np.array([0, 1, 2]), busy, 5.0, nl)
    assert r["members"] == 3 and r["streams"] == 3
    assert r["per_chi"]["16"]["gate_steps"] == 2 * 2 * nl
    assert r["per_chi"]["64"]["gate_steps"] == 2 * 2 * nl + 2 * (nl - 1)
    assert abs(r["per_chi"]["16"]["rate_on_its_streams"] - 4 * nl / 2e-3) < 1e-6
    assert abs(r["utilisation_busy_over_streams_x_elapsed"] - 12.0 / 15.0) < 1e-12
    tot = 4 * nl + 4 * nl + 2 * (nl - 1)
    assert abs(r["rate_all"] - tot / 5e-3) < 1e-6
