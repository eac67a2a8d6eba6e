"""GPU parity of whole trajectories (apply_layer + expect through the C ABI) with the
oracle on the same seeded inputs:

* state-independent unravellings (ORTHOGONAL / FIXED): branch choices identical and
  per-trajectory observables within 1e-10 (FP64) / 1e-4 (FP32-bulk) of the oracle
  statevector (exact bond dimension) or oracle MPS (truncated);
* the optimal unravelling: the oracle replays the GPU's recorded mixings, checking each one
  for optimality on its own reduced state and completeness, and must reproduce the GPU's
  branch choices and observables.
"""
import numpy as np
import pytest

from oracle import sv as osv
from oracle import unravel as OU
from paper_2508_05745_amd import inputs as I

from gpu_util import oracle_obs_mps, oracle_obs_sv, recorded_events, run_gpu

pytestmark = pytest.mark.gpu


def _circuit(n, depth, seed, channel, idle=False):
    return I.brickwork(n, depth, seed=seed, channel=channel, idle_noise=idle)


@pytest.mark.parametrize("prec,tol", [(1, 1e-10), (0, 1e-4)])
@pytest.mark.parametrize("mode", [0, 1])
def test_fixed_unravelling_exact_bond(prec, tol, mode):
    from paper_2508_05745_amd import mpsb as M
    c = _circuit(6, 5, 21, I.depolarizing(0.1), idle=True)
    fixed = OU.H4.real if mode == 1 else None
    out = run_gpu(c, 8, 24, 77, prec, mode, fixed, record=True)
    for t in range(24):
        rec = []
        ref = oracle_obs_sv(c, t, 77, mode, fixed, record=rec)
        _, js = recorded_events(c, out, t)
        assert js == [r["j"] for r in rec], t
        assert np.abs(out["per_traj"][t] - ref).max() < tol, (t, np.abs(out["per_traj"][t] - ref).max())


@pytest.mark.parametrize("prec,tol,gap", [(1, 1e-10, 1e-9), (0, 1e-4, 1e-4)])
def test_optimal_unravelling_replay(prec, tol, gap):
    c = _circuit(8, 6, 22, I.depolarizing(0.05))
    out = run_gpu(c, 16, 32, 78, prec, 3, record=True)
    for t in range(32):
        ws, js = recorded_events(c, out, t)
        rp = osv.Replay(ws)
        rec = []
        ref = oracle_obs_sv(c, t, 78, 3, replay=rp, record=rec)
        assert js == [r["j"] for r in rec], t
        assert rp.max_incomplete < 1e-10
        assert rp.max_gap < gap, rp.max_gap
        assert np.abs(out["per_traj"][t] - ref).max() < tol


def test_optimal_unravelling_ad_dephasing_idle_replay():
    c = _circuit(7, 5, 23, I.compose(I.amplitude_damping(0.05), I.dephasing(0.05)), idle=True)
    out = run_gpu(c, 8, 16, 79, 1, 3, record=True)
    for t in range(16):
        ws, js = recorded_events(c, out, t)
        rp = osv.Replay(ws)
        rec = []
        ref = oracle_obs_sv(c, t, 79, 3, replay=rp, record=rec)
        assert js == [r["j"] for r in rec]
        assert rp.max_gap < 1e-9 and rp.max_incomplete < 1e-10
        assert np.abs(out["per_traj"][t] - ref).max() < 1e-10


@pytest.mark.parametrize("prec,tol", [(1, 1e-10), (0, 1e-4)])
def test_truncated_trajectories_match_oracle_mps(prec, tol):
    """chi below the exact bond dimension: same truncation (top-chi Schmidt subspace) on
    both sides, state-independent unravelling, per-trajectory observables and discarded
    weights."""
    c = _circuit(10, 8, 24, I.depolarizing(0.02))
    chi = 4
    out = run_gpu(c, chi, 12, 80, prec, 0, record=True)
    for t in range(12):
        ref, eps = oracle_obs_mps(c, chi, t, 80, 0)
        assert np.abs(out["per_traj"][t] - ref).max() < tol
        gd = []
        for l in range(c.depth):
            order = [q for kind, q in osv.sweep_ops(c, l) if kind == "gate"]
            for q in order:
                gd.append(out["disc"][l][t, (q - l % 2) // 2])
        assert np.abs(np.array(gd) - np.array(eps)).max() < (1e-10 if prec == 1 else 1e-5)


def test_replay_inputs_follow_a_recorded_run():
    """apply_layer with replay inputs: an FP64 run fed its own recorded mixings and branches
    (or only the branches) reproduces itself bit for bit; an FP32-bulk run fed the FP64 run's
    decisions takes the same branches and stays within 1e-4 of it per trajectory (the paired
    comparison of the two precisions)."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    c = I.brickwork(10, 8, seed=45, channel=I.depolarizing(0.05))
    T, chi = 64, 16

    def run(prec, w_in=None, b_in=None):
        b = M.Batch(T, c.n, chi, prec, 13)
        b.set_circuit(c, M.OPTIMAL)
        w = torch.zeros((T, c.n, 4, 4), dtype=torch.complex128, device="cuda")
        br = torch.zeros((T, c.n), dtype=torch.int32, device="cuda")
        ws, brs = [], []
        for l in range(c.depth):
            b.apply_layer(l, branch=br, w_record=w,
                          w_in=None if w_in is None else w_in[l], branch_in=None if b_in is None else b_in[l])
            ws.append(w.clone())
            brs.append(br.clone())
        _, _, pt = b.expect()
        b.sync()
        out = (pt.cpu().numpy(), ws, brs)
        b.close()
        return out

    ref, ws, brs = run(1)
    same, ws2, brs2 = run(1, ws, brs)
    assert np.array_equal(same, ref)
    assert all(torch.equal(a, b) for a, b in zip(brs, brs2))
    only_b, _, _ = run(1, None, brs)
    assert np.array_equal(only_b, ref)
    f32, _, brs32 = run(0, ws, brs)
    assert all(torch.equal(a, b) for a, b in zip(brs, brs32))
    err = np.abs(f32 - ref).max()
    print(f"FP32-bulk replay of the FP64 run: max |d<O>| = {err:.2e}", flush=True)
    assert err < 1e-4
