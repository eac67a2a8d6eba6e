"""Whole-layer HIP graphs and mixed batches.

* Graph replay: with graphs on, a layer signature's first occurrence runs directly, the
  second is captured and later ones replay the graph; the state buffers must equal those of
  a run with graphs off, bit for bit, after every layer (eager torch work and device
  synchronisations between the replays).
* Mixed batches (trajectories of different widths, depths, bond dimensions and noise
  strengths, gates from a shared pool): every trajectory, replayed by the oracle on its own
  circuit with the GPU's recorded mixings, matches branch for branch and in its
  observables; the graph-replayed run (no records) gives the recorded run's observables bit
  for bit.
"""
import numpy as np
import pytest

from oracle import mps as omps
from oracle import sv as osv
from paper_2508_05745_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("record", [False, True])
@pytest.mark.parametrize("prec", [1, 0])
def test_graph_replays_match_direct_runs(prec, record):
    """record: both runs write the discarded weights, branches and mixings of every layer
    into the same output buffers each layer (the addresses are part of the graph's
    signature, so the graph run captures and replays its records too)."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    c = I.brickwork(10, 8, seed=41, channel=I.depolarizing(0.05), idle_noise=True)
    T = 64
    a = M.Batch(T, c.n, 16, prec, 5)
    b = M.Batch(T, c.n, 16, prec, 5)
    a.set_circuit(c, M.OPTIMAL)
    b.set_circuit(c, M.OPTIMAL)
    b.set_graphs(False)

    def bufs():
        if not record:
            return dict()
        return dict(discarded=torch.zeros((T, c.n // 2), dtype=torch.float64, device="cuda"),
                    branch=torch.zeros((T, c.n), dtype=torch.int32, device="cuda"),
                    w_record=torch.zeros((T, c.n, 4, 4), dtype=torch.complex128, device="cuda"))
    ra, rb = bufs(), bufs()
    for l in range(c.depth):
        a.apply_layer(l, **ra)
        b.apply_layer(l, **rb)
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        _ = (x * x).sum().item()
        torch.cuda.synchronize()
        assert torch.equal(a.state, b.state), l
        for k in ra:
            assert torch.equal(ra[k], rb[k]), (l, k)
        if record and l > 0:
            assert bool((ra["branch"] >= 0).any()), l
    ma, _, pa = a.expect()
    mb, _, pb = b.expect()
    assert torch.equal(pa, pb)
    a.sync()
    b.sync()
    a.close()
    b.close()


def _run_mixed(mc, seed, prec, record, verbose=False):
    import torch

    from paper_2508_05745_amd import mpsb as M
    b = M.Batch(mc.n_traj, mc.widths, mc.chis, prec, seed)
    b.set_circuit(mc, M.OPTIMAL)
    T, W = mc.n_traj, mc.n
    w = torch.zeros((T, W, 4, 4), dtype=torch.complex128, device="cuda") if record else None
    br = torch.zeros((T, W), dtype=torch.int32, device="cuda") if record else None
    ws, brs = [], []
    for l in range(mc.depth):
        b.apply_layer(l, branch=br, w_record=w)
        if verbose:
            print(f"layer {l} queued", flush=True)
        if record:
            ws.append(w.cpu().numpy())
            brs.append(br.cpu().numpy())
    _, _, pt = b.expect()
    b.sync()
    out = dict(per_traj=pt.cpu().numpy(), w=ws, branch=brs)
    b.close()
    return out


def _replay_mixed(mc, seed, out, t, tol, u):
    c = mc.trajectory_circuit(t)
    ws, js = [], []
    for l in range(c.depth):
        for kind, q in osv.sweep_ops(c, l):
            for x in osv.event_qubits(c, l, kind, q):
                ws.append(out["w"][l][t, x].T.copy())
                js.append(int(out["branch"][l][t, x]))
    rp = osv.Replay(ws)
    rec, spectra = [], []
    m, _ = omps.trajectory(c, int(mc.chis[t]), t, seed, mode=3, record=rec, replay=rp, spectra=spectra)
    zi, zz = omps.z_expectations(m)
    ref = np.concatenate([zi, zz])
    assert js == [r["j"] for r in rec], t
    assert rp.max_incomplete < 1e-10 and rp.max_gap < (1e-9 if u < 1e-10 else 1e-4), (t, rp.max_gap)
    got = out["per_traj"][t]
    nobs = 2 * c.n - 1
    assert np.isnan(got[nobs:]).all()
    err = np.abs(got[:nobs] - ref).max()
    print(f"traj {t} (width {c.n}, depth {c.depth}, chi {mc.chis[t]}): max |d<O>| {err:.1e}, tol {tol:.1e}",
          flush=True)
    assert err < tol, (t, err, tol)


@pytest.mark.parametrize("prec,tol,u", [(1, 1e-10, 2.0 ** -53), (0, 1e-4, 2.0 ** -24)])
def test_mixed_batch_replay_and_graphs(prec, tol, u):
    mc = I.mixed_brickwork(40, seed=11, widths=(5, 10), depths=(3, 7), chis=(4, 8, 16), pool_size=64)
    rec = _run_mixed(mc, 23, prec, True)
    for t in range(mc.n_traj):
        _replay_mixed(mc, 23, rec, t, tol, u)
    fast = _run_mixed(mc, 23, prec, False)
    assert np.array_equal(np.nan_to_num(fast["per_traj"], nan=7.0), np.nan_to_num(rec["per_traj"], nan=7.0))


def test_mixed_workload_sampled():
    """The mixed-batch workload's distributions (chi 16..128, depolarizing 0.005..0.03,
    2^16-gate pool) with widths 24..32 and depths 16..20 at 256 trajectories, FP32-bulk;
    one sampled trajectory of every chi class replayed by the oracle."""
    mc = I.mixed_brickwork(256, seed=1003, widths=(24, 32), depths=(16, 20))
    rec = _run_mixed(mc, 2003, 0, True, verbose=True)
    chis = mc.chis
    sample = [int(np.flatnonzero(chis == c)[0]) for c in (16, 32, 64, 128)]
    for t in sample:
        _replay_mixed(mc, 2003, rec, t, 1e-4, 2.0 ** -24)
    assert np.isfinite(rec["per_traj"][:, 0]).all()


@pytest.mark.parametrize("prec", [1, 0])
def test_trajectory_offset_waves_reproduce_one_batch(prec):
    """A run of T trajectories done as two memory waves (batches of T/2 with trajectory
    offsets 0 and T/2) draws the same branches and reaches the same states as one batch of T:
    per-trajectory observables and recorded branches equal bit for bit."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    c = I.brickwork(10, 8, seed=43, channel=I.depolarizing(0.05))
    T = 64

    def run(n, off):
        b = M.Batch(n, c.n, 16, prec, 9, traj_offset=off)
        b.set_circuit(c, M.OPTIMAL)
        br = torch.zeros((n, c.n), dtype=torch.int32, device="cuda")
        brs = []
        for l in range(c.depth):
            b.apply_layer(l, branch=br)
            brs.append(br.cpu().numpy().copy())
        _, _, pt = b.expect()
        b.sync()
        out = (pt.cpu().numpy(), np.stack(brs, axis=1))
        b.close()
        return out

    whole = run(T, 0)
    a = run(T // 2, 0)
    b = run(T // 2, T // 2)
    assert np.array_equal(np.concatenate([a[1], b[1]]), whole[1])
    assert np.array_equal(np.concatenate([a[0], b[0]]), whole[0])


def test_mixed_schedule_timing():
    """Schedule timing (mps_profile bit 1) of a mixed batch: the members partition the
    trajectories in order, every timed layer is counted, members with work have positive busy
    time on one of at most four streams, the busy times fit in four streams' share of the
    elapsed time, and the timed run (direct launches, streams dealt round-robin) gives the
    untimed run's observables bit for bit."""
    from paper_2508_05745_amd import mpsb as M
    mc = I.mixed_brickwork(40, seed=11, widths=(5, 10), depths=(3, 7), chis=(4, 8, 16), pool_size=64)
    plain = _run_mixed(mc, 23, 0, False)
    b = M.Batch(mc.n_traj, mc.widths, mc.chis, 0, 23)
    b.set_circuit(mc, M.OPTIMAL)
    b.profile(2)
    for l in range(mc.depth):
        b.apply_layer(l)
    first, count, stream, busy, elapsed, layers = b.schedule_read()
    _, _, pt = b.expect()
    b.sync()
    b.profile(0)
    b.close()
    runs = 1 + int(np.count_nonzero((np.diff(mc.widths) != 0) | (np.diff(mc.chis) != 0)))
    assert len(first) == runs
    assert first[0] == 0 and np.array_equal(first[1:], np.cumsum(count)[:-1]) and count.sum() == mc.n_traj
    assert layers == mc.depth and elapsed > 0
    assert (busy > 0).all() and ((stream >= 0) & (stream < 4)).all()
    assert busy.sum() <= 4 * elapsed * 1.05 + 0.5
    print(f"{runs} members, {layers} layers: busy {busy.sum():.2f} ms over {elapsed:.2f} ms elapsed", flush=True)
    assert np.array_equal(np.nan_to_num(pt.cpu().numpy(), nan=7.0), np.nan_to_num(plain["per_traj"], nan=7.0))


@pytest.mark.parametrize("prec", [1, 0])
def test_mixed_batch_mean_and_m2(prec):
    """expect on a mixed batch: mean and M2 in the widest trajectory's layout over the
    trajectories that have each observable (<Z_i>: width > i, <Z_i Z_(i+1)>: width > i + 1),
    against a two-pass NumPy mean / M2 of the per-trajectory rows (each row in its own width's
    layout); a second call (without rows, after the first sweep has moved the centres, so the
    state is in another gauge) agrees to rounding."""
    from paper_2508_05745_amd import mpsb as M
    mc = I.mixed_brickwork(40, seed=11, widths=(5, 10), depths=(3, 7), chis=(4, 8, 16), pool_size=64)
    b = M.Batch(mc.n_traj, mc.widths, mc.chis, prec, 23)
    b.set_circuit(mc, M.OPTIMAL)
    for l in range(mc.depth):
        b.apply_layer(l)
    mean, m2, pt = b.expect()
    mean2, m22, _ = b.expect(per_traj=False)
    b.sync()
    b.close()
    mean, m2, pt = mean.cpu().numpy(), m2.cpu().numpy(), pt.cpu().numpy()
    tol = 1e-12 if prec == 1 else 1e-5
    fin = np.isfinite(mean)
    assert np.array_equal(fin, np.isfinite(mean2.cpu().numpy()))
    assert np.abs(mean[fin] - mean2.cpu().numpy()[fin]).max() < tol
    assert np.abs(m2[fin] - m22.cpu().numpy()[fin]).max() < tol * mc.n_traj
    W = mc.n
    for k in range(2 * W - 1):
        vals = []
        for t in range(mc.n_traj):
            n = int(mc.widths[t])
            if k < W and k < n:
                vals.append(pt[t, k])
            elif k >= W and k - W < n - 1:
                vals.append(pt[t, n + k - W])
        if not vals:
            assert np.isnan(mean[k]) and np.isnan(m2[k]), k
            continue
        v = np.array(vals)
        assert abs(mean[k] - v.mean()) < 1e-13, k
        assert abs(m2[k] - ((v - v.mean()) ** 2).sum()) < 1e-12 * max(1.0, len(v)), k
