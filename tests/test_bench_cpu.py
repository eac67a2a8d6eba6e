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
