"""GPU observables against the exact density matrix (statistical agreement of trajectory
averages), FP32-bulk vs FP64 statistics, and the edge entry points sample_kraus /
mps_truncate through the C ABI."""
import numpy as np
import pytest

from oracle import dm as odm
from oracle import mps as omps
from oracle import unravel as OU
from paper_2508_05745_amd import inputs as I

from gpu_util import oracle_obs_mps, run_gpu

pytestmark = pytest.mark.gpu


def _zscores(out, exact):
    n_traj = out["per_traj"].shape[0]
    se = np.sqrt(out["m2"] / (n_traj - 1) / n_traj) + 1e-15
    return np.abs(out["mean"] - exact) / se


@pytest.mark.parametrize("prec", [1, 0])
def test_small_exact_config_vs_density_matrix(prec):
    """10 qubits, depth 10, depolarizing 0.01 after each gate, chi=32 (exact), 1000
    trajectories, optimal unravelling: every <Z_i>, <Z_i Z_i+1> within 4 sigma of the exact
    density matrix, and the chi^2 of the 19 z-scores consistent with 19 dof."""
    wl = I.config_small_exact()
    c = wl.circuit
    out = run_gpu(c, wl.chi, wl.n_traj, wl.seed, prec, 3)
    zi, zz = odm.z_expectations(odm.run(c), c.n)
    z = _zscores(out, np.concatenate([zi, zz]))
    assert z.max() < 4.0, z
    assert np.sum(z ** 2) < 19 + 6 * np.sqrt(2 * 19)
    # mean and M2 agree with the per-trajectory values
    pt = out["per_traj"]
    assert np.allclose(out["mean"], pt.mean(0), atol=1e-12)
    assert np.allclose(out["m2"], ((pt - pt.mean(0)) ** 2).sum(0), rtol=1e-9, atol=1e-12)


def test_unravelling_independence_of_the_average():
    """Different unravellings (orthogonal, Haar-optimal fixed, optimal) give the same
    average state: the three trajectory averages agree with the exact state within 4 sigma."""
    c = I.brickwork(8, 6, seed=31, channel=I.depolarizing(0.1))
    zi, zz = odm.z_expectations(odm.run(c), c.n)
    ex = np.concatenate([zi, zz])
    for mode, fixed in ((0, None), (1, OU.H4.real), (3, None)):
        out = run_gpu(c, 16, 2000, 91 + mode, 1, mode, fixed)
        assert _zscores(out, ex).max() < 4.0, mode


def test_fp32_bulk_vs_fp64_statistics_ad_dephasing():
    """Amplitude damping + dephasing on every qubit every layer (idle qubits included),
    truncating chi: FP32-bulk and FP64 trajectory averages agree within their combined
    statistical error; per-trajectory FP32 vs FP64 differences are reported, not gated
    (the optimal decomposition is not unique, so paired trajectories can branch apart)."""
    ch = I.compose(I.amplitude_damping(0.005), I.dephasing(0.005))
    c = I.brickwork(16, 10, seed=32, channel=ch, idle_noise=True)
    a = run_gpu(c, 8, 1024, 92, 1, 3)
    b = run_gpu(c, 8, 1024, 92, 0, 3)
    se = np.sqrt(a["m2"] / 1023 / 1024 + b["m2"] / 1023 / 1024) + 1e-15
    assert (np.abs(a["mean"] - b["mean"]) / se).max() < 4.5


def test_sample_kraus_forced_and_drawn():
    import torch

    from oracle import rng as orng
    from oracle import sv as osv
    from paper_2508_05745_amd import mpsb as M
    c = I.brickwork(5, 2, seed=33, channel=I.amplitude_damping(0.3))
    T = 8
    b = M.Batch(T, 5, 8, M.FP64, 44)
    b.set_circuit(c, M.ORTHOGONAL)
    b.apply_layer(0)
    b.apply_layer(1)
    br = torch.zeros(T, dtype=torch.int32, device="cuda")
    p = torch.zeros((T, 4), dtype=torch.float64, device="cuda")
    # drawn event on qubit 2 keyed by (traj, layer 7, qubit 2)
    b.sample_kraus(2, 0, M.ORTHOGONAL, 7, branch=br, p=p)
    _, _, pt = b.expect()
    b.sync()
    for t in range(T):
        psi = osv.trajectory(c, t, 44, mode=0)
        rq = osv.reduced_one(psi, 5, 2)
        ps = np.array([np.vdot(osv.apply_one(psi, 5, 2, k), osv.apply_one(psi, 5, 2, k)).real
                       for k in c.kraus(0)] + [0.0, 0.0])
        assert np.abs(ps - p[t].cpu().numpy()).max() < 1e-12
        j = orng.sample_branch(ps, orng.uniform(44, t, 7, 2))
        assert j == int(br[t])
        psi2 = osv.apply_one(psi, 5, 2, c.kraus(0)[j]) / np.sqrt(ps[j])
        zi, zz = osv.z_expectations(psi2, 5)
        assert np.abs(np.concatenate([zi, zz]) - pt[t].cpu().numpy()).max() < 1e-10
    # a forced zero-probability branch fails before touching the state
    forced = np.full(T, 3, dtype=np.int32)       # operator 3 does not exist (p = 0)
    with pytest.raises(M.MpsbError) as e:
        b.sample_kraus(2, 0, M.ORTHOGONAL, 8, forced=forced)
    assert e.value.code == M.ENUM
    _, _, pt2 = b.expect()
    b.sync()
    assert np.abs(pt2.cpu().numpy() - pt.cpu().numpy()).max() < 1e-13
    b.close()


@pytest.mark.parametrize("prec,tol", [(1, 1e-10), (0, 1e-4)])
def test_truncate_entry_point(prec, tol):
    """Noiseless circuit run exactly, then one truncation sweep to chi=3: observables equal
    the oracle's exact state truncated bond by bond (left to right) with SVDs."""
    from paper_2508_05745_amd import mpsb as M
    import torch
    c = I.noiseless_copy(I.brickwork(8, 6, seed=34, channel=I.depolarizing(0.1)))
    T = 4
    b = M.Batch(T, 8, 16, prec, 1)
    b.set_circuit(c, M.ORTHOGONAL)
    for l in range(c.depth):
        b.apply_layer(l)
    disc = torch.zeros(T, dtype=torch.float64, device="cuda")
    b.truncate(3, disc)
    _, _, pt = b.expect()
    b.sync()
    m, _ = omps.trajectory(c, 16, 0, 1, mode=0)
    tot = 0.0
    m.move_centre(0)
    for k in range(c.n - 1):
        m.move_centre(k)
        th = np.einsum("sab,tbc->stac", m.t[k], m.t[k + 1])
        dl, dr = th.shape[2], th.shape[3]
        mat = th.transpose(0, 2, 1, 3).reshape(2 * dl, 2 * dr)
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
        d = min(3, s.size)
        tot += float(np.sum(s[d:] ** 2) / np.sum(s ** 2))
        s = s[:d] / np.sqrt(np.sum(s[:d] ** 2))
        m.t[k] = u[:, :d].reshape(2, dl, d)
        m.t[k + 1] = (s[:, None] * vh[:d]).reshape(d, 2, dr).transpose(1, 0, 2)
        m.centre = k + 1
    zi, zz = omps.z_expectations(m)
    ref = np.concatenate([zi, zz])
    for t in range(T):
        assert np.abs(pt[t].cpu().numpy() - ref).max() < tol
        assert abs(float(disc[t]) - tot) < (1e-10 if prec == 1 else 1e-5)
    b.close()
