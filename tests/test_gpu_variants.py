"""Variants of the method through the library, against the oracle on the same seeded inputs:

* Born sampling from the trajectories (Lemma "Output distribution sampling from trajectory
  sampling"): the same counter draws give the same bitstrings as the oracle's sampler on the
  same trajectory states, and one sample per trajectory follows <x|rho|x> of the exact noisy
  state;
* global layering (gates and noise of a layer with 2 chi intermediate bonds, then one
  truncation sweep to chi): per-trajectory observables and discarded weights against the
  oracle's global layering.
"""
import math

import numpy as np
import pytest

from oracle import dm as odm
from oracle import mps as omps
from paper_2508_05745_amd import inputs as I

pytestmark = pytest.mark.gpu


def _batch(c, chi, T, prec, seed, mode):
    from paper_2508_05745_amd import mpsb as M
    b = M.Batch(T, c.n, chi, prec, seed)
    b.set_circuit(c, mode)
    return b


@pytest.mark.parametrize("prec", [1, 0])
def test_born_samples_match_oracle(prec):
    c = I.brickwork(8, 6, seed=71, channel=I.depolarizing(0.05))
    T, S = 16, 8
    b = _batch(c, 16, T, prec, 97, 0)
    for l in range(c.depth):
        b.apply_layer(l)
    bits = b.sample_bitstrings(S, 123).cpu().numpy()
    b.sync()
    b.close()
    same, total = 0, 0
    for t in range(T):
        m, _ = omps.trajectory(c, 16, t, 97, mode=0)
        ref, _ = omps.born_sample(m, S, 123, t)
        same += int((bits[t] == ref).all(axis=1).sum())
        total += S
    print(f"identical bitstrings: {same} of {total}", flush=True)
    if prec == 1:
        assert same == total
    else:
        assert same >= total - 2          # FP32 products can move a draw that lies within ~1e-7 of a boundary


def test_born_samples_follow_the_mixed_state():
    """One sample from each of 8192 trajectories (6 qubits, depth 6, amplitude damping 0.2,
    optimal unravelling, FP64): chi^2 of the 64 outcome counts against <x|rho|x>."""
    from paper_2508_05745_amd import mpsb as M
    c = I.brickwork(6, 6, seed=72, channel=I.amplitude_damping(0.2))
    T = 8192
    b = _batch(c, 8, T, 1, 98, M.OPTIMAL)
    for l in range(c.depth):
        b.apply_layer(l)
    bits = b.sample_bitstrings(1, 7).cpu().numpy()[:, 0, :]
    b.sync()
    b.close()
    idx = (bits.astype(np.int64) * (1 << np.arange(5, -1, -1))).sum(1)
    counts = np.bincount(idx, minlength=64)
    exp = np.real(np.diag(odm.run(c))) * T
    keep = exp > 5
    chi2 = float(((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum())
    print(f"chi^2 {chi2:.1f} over {keep.sum()} outcomes", flush=True)
    assert chi2 < keep.sum() + 6 * math.sqrt(2 * keep.sum())


@pytest.mark.parametrize("prec,tol,dtol", [(1, 1e-10, 1e-10), (0, 1e-4, 1e-5)])
def test_global_layering_matches_oracle(prec, tol, dtol):
    import torch
    c = I.brickwork(10, 6, seed=73, channel=I.depolarizing(0.05))
    chi, T = 4, 8
    b = _batch(c, 2 * chi, T, prec, 99, 0)
    d = torch.zeros(T, dtype=torch.float64, device="cuda")
    disc = []
    for l in range(c.depth):
        b.apply_layer_global(l, chi, d)
        disc.append(d.cpu().numpy().copy())
    _, _, pt = b.expect()
    pt = pt.cpu().numpy()
    b.sync()
    b.close()
    for t in range(T):
        m, eps = omps.trajectory_global(c, chi, t, 99, mode=0)
        zi, zz = omps.z_expectations(m)
        assert np.abs(pt[t] - np.concatenate([zi, zz])).max() < tol, t
        for l in range(c.depth):
            assert abs(disc[l][t] - sum(eps[l])) < dtol, (t, l)
    assert max(float(x.max()) for x in disc) > 1e-4          # the sweeps truncate
