"""Trotterised Lindbladian workload (Sec. "Time-independent Lindbladian systems") through the
library, against the oracle on the same model (each side builds its own circuit: the
library's mps_trotter_gate / mps_jump_channel, the oracle's scipy construction):

* the library's gates and Choi-derived Kraus operators equal the oracle's (same phase
  convention), including the paper's dephasing / amplitude-damping identifications;
* per-trajectory parity under the optimal unravelling (the oracle replays the GPU's recorded
  mixings on its own circuit), FP64 and FP32-bulk;
* the trajectory average of the Fig.-6 Hamiltonian with amplitude damping against the exact
  density matrix of the Trotterised circuit (4 sigma per observable, chi^2 over all).
"""
import math

import numpy as np
import pytest

from oracle import dm as odm
from oracle import lindblad as OL
from oracle import sv as osv
from paper_2508_05745_amd import inputs as I

from gpu_util import oracle_obs_sv, recorded_events, run_gpu

pytestmark = pytest.mark.gpu

SM = np.array([[0, 1], [0, 0]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)


def test_library_constructors_match_oracle():
    from paper_2508_05745_amd import mpsb as M
    rng = np.random.default_rng(11)
    for _ in range(20):
        g = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        h = 0.5 * (g + g.conj().T)
        dt = rng.uniform(0.001, 0.5)
        assert np.abs(M.trotter_gate(h, dt) - OL.trotter_gate(h, dt)).max() < 1e-13
    cases = [[(SM, 0.8)], [(P0, 1.7)], [(SM, 0.5), (P0, 0.3)]]
    cases += [[(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)), rng.uniform(0.1, 2.0))]
              for _ in range(10)]
    for jumps in cases:
        tau = float(rng.uniform(0.005, 0.4))
        k = M.jump_channel(jumps, tau)
        ko = OL.jump_kraus(jumps, tau)
        assert k.shape == ko.shape
        assert np.abs(k - ko).max() < 1e-12
    # the paper's identifications, through the library
    k = M.jump_channel([(SM, 2.0)], 0.05)
    gad = 1.0 - math.exp(-2.0 * 0.05)
    assert np.abs(k - I.amplitude_damping(gad)).max() < 1e-14
    k = M.jump_channel([(P0, 2.0)], 0.05)
    assert np.abs(k - I.dephasing(1.0 - math.exp(-0.05))).max() < 1e-14


@pytest.mark.parametrize("prec,tol,gap", [(1, 1e-10, 1e-9), (0, 1e-4, 1e-4)])
def test_lindblad_trajectories_replay(prec, tol, gap):
    from paper_2508_05745_amd import mpsb as M
    m = I.lindblad_random_ti(n=8, steps=4, dt=0.05, gamma_ad=0.05, seed=7)
    cg, co = M.lindblad_circuit(m), OL.circuit(m)
    out = run_gpu(cg, 16, 16, 95, prec, M.OPTIMAL, record=True)
    for t in range(16):
        ws, js = recorded_events(cg, out, t)
        rp = osv.Replay(ws)
        rec = []
        ref = oracle_obs_sv(co, t, 95, 3, replay=rp, record=rec)
        assert js == [r["j"] for r in rec], t
        assert rp.max_incomplete < 1e-10 and rp.max_gap < gap, rp.max_gap
        assert np.abs(out["per_traj"][t] - ref).max() < tol


def test_heisenberg_average_vs_trotterised_density_matrix():
    """10 qubits, the Fig.-6 Hamiltonian, dt = 0.05, 8 Trotter steps, amplitude damping 0.05 per
    layer, 4096 trajectories (FP64, optimal unravelling, exact bond dimension)."""
    from paper_2508_05745_amd import mpsb as M
    m = I.lindblad_heisenberg(n=10, steps=8, dt=0.05, gamma_ad=0.05)
    out = run_gpu(M.lindblad_circuit(m), 32, 4096, 96, 1, M.OPTIMAL)
    zi, zz = odm.z_expectations(odm.run(OL.circuit(m)), m.n)
    ref = np.concatenate([zi, zz])
    pt = out["per_traj"]
    se = pt.std(0, ddof=1) / math.sqrt(pt.shape[0]) + 1e-300
    z = np.abs(pt.mean(0) - ref) / se
    print(f"max z {z.max():.2f}, chi^2 {np.sum(z ** 2):.1f} over {z.size}", flush=True)
    assert z.max() < 4.5, z
    assert np.sum(z ** 2) < z.size + 6 * math.sqrt(2 * z.size)
