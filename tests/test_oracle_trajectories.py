"""Pins of the oracle's density-matrix, statevector and MPS trajectory code (no GPU)."""
import numpy as np
import pytest

from oracle import dm, kraus_tree, mps, sv, unravel as U
from paper_2508_05745_amd import inputs as I


def test_density_matrix_is_a_state():
    c = I.brickwork(5, 4, seed=3, channel=I.depolarizing(0.1), idle_noise=True)
    rho = dm.run(c)
    assert abs(np.trace(rho) - 1) < 1e-13
    assert np.allclose(rho, rho.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(rho).min() > -1e-13


def test_density_matrix_two_qubit_hand_case():
    """One gate then depolarizing on both qubits: (D x D)(G|00><00|G^dag) with the
    depolarizing map D(X) = (1-p) X + p Tr_q(X) I/2 written out."""
    p = 0.2
    c = I.brickwork(2, 1, seed=4, channel=I.depolarizing(p))
    g = c.gate(0, 0)
    psi = g[:, 0]
    r = np.outer(psi, psi.conj()).reshape(2, 2, 2, 2)
    r = (1 - p) * r + p * np.einsum("ab,cxcy->axby", np.eye(2) / 2, r)
    r = (1 - p) * r + p * np.einsum("xy,acbc->axby", np.eye(2) / 2, r)
    assert np.allclose(dm.run(c), r.reshape(4, 4), atol=1e-14)


@pytest.mark.parametrize("mode", [U.MODE_OPTIMAL, U.MODE_ORTHOGONAL, U.MODE_FIXED])
def test_kraus_tree_average_is_exact_state(mode):
    """Without approximation the Kraus-tree average equals rho for any unravelling."""
    fixed = U.H4.real if mode == U.MODE_FIXED else None
    c = I.brickwork(3, 2, seed=5, channel=I.depolarizing(0.1))
    assert np.abs(kraus_tree.average_state(c, mode, fixed) - dm.run(c)).max() < 1e-13
    c2 = I.brickwork(3, 2, seed=6, channel=I.compose(I.amplitude_damping(0.2),
                                                    I.dephasing(0.3)), idle_noise=True)
    if mode != U.MODE_FIXED:
        assert np.abs(kraus_tree.average_state(c2, mode) - dm.run(c2)).max() < 1e-13


@pytest.mark.parametrize("mode", [U.MODE_ORTHOGONAL, U.MODE_OPTIMAL])
def test_untruncated_mps_equals_statevector(mode):
    """Same seeds, no truncation: identical branch choices, fidelity 1 to 1e-12 and
    equal observables (OPTIMAL: the statevector replays the MPS's mixings, which it checks
    for optimality on its own reduced states)."""
    c = I.brickwork(8, 6, seed=7, channel=I.compose(I.amplitude_damping(0.05),
                                                   I.dephasing(0.05)), idle_noise=True)
    for traj in range(3):
        rec = []
        m, eps = mps.trajectory(c, 16, traj, 99, mode=mode, record=rec)
        rp = sv.Replay([r["W"] for r in rec]) if mode == U.MODE_OPTIMAL else None
        rec2 = []
        psi = sv.trajectory(c, traj, 99, mode=mode, record=rec2, replay=rp)
        v = m.to_vector()
        assert [a["j"] for a in rec] == [b["j"] for b in rec2]
        assert 1 - abs(np.vdot(psi, v)) ** 2 < 1e-12
        assert max(eps) < 1e-14
        zi, zz = sv.z_expectations(psi, 8)
        zi2, zz2 = mps.z_expectations(m)
        assert np.abs(zi - zi2).max() < 1e-12 and np.abs(zz - zz2).max() < 1e-12
        if rp is not None:
            assert rp.max_gap < 1e-12 and rp.max_incomplete < 1e-12


def test_norm_preserved_and_truncation_weight():
    c = I.brickwork(10, 8, seed=8, channel=I.depolarizing(0.02))
    m, eps = mps.trajectory(c, 4, 0, 5)
    assert abs(np.linalg.norm(m.to_vector()) - 1) < 1e-12
    assert max(eps) > 1e-6
    assert max(m.bond_dims()) <= 4


def _truncating_step(n, q, chi, seed):
    """An entangled n-qubit trajectory state (exact, noisy, several layers), then one
    gate-step on (q, q+1) twice from the same state and seeds: untruncated (the state before
    the approximation) and truncated to chi.  Returns (psi_full, psi_trunc, eps)."""
    import copy
    c = I.brickwork(n, 8, seed=seed, channel=I.depolarizing(0.05))
    layer = 7
    m, _ = mps.trajectory(c, 2 ** n, 0, seed, layers=layer)
    full, trunc = copy.deepcopy(m), copy.deepcopy(m)
    eps_full = mps.gate_step(full, layer, q, c, 2 ** n, 0, seed, U.MODE_OPTIMAL)
    eps = mps.gate_step(trunc, layer, q, c, chi, 0, seed, U.MODE_OPTIMAL)
    assert eps_full < 1e-14
    return full.to_vector(), trunc.to_vector(), eps


@pytest.mark.parametrize("n,q,chi", [(8, 3, 3), (8, 3, 7), (7, 2, 2), (6, 1, 1)])
def test_truncation_keeps_top_schmidt_values(n, q, chi):
    """Truncation (eq. MPS_truncation_error, Eckart-Young): the discarded weight is the sum of
    the squared Schmidt values of the *full* state across the cut beyond the chi largest
    (Schmidt values from the SVD of the whole state vector reshaped at the cut, not from the
    oracle's local two-site tensor), and the truncated state is the renormalised projection:
    ||psi - sqrt(1 - eps) psi_trunc||^2 = eps and |<psi|psi_trunc>|^2 = 1 - eps."""
    psi, pt, eps = _truncating_step(n, q, chi, seed=31 + n + chi)
    s = np.linalg.svd(psi.reshape(2 ** (q + 1), -1), compute_uv=False)
    assert s[chi] > 1e-3 * s[0]                       # the cut discards real weight
    assert eps == pytest.approx(float(np.sum(s[chi:] ** 2)), rel=1e-10, abs=1e-15)
    assert abs(np.linalg.norm(pt) - 1) < 1e-13
    ov = np.vdot(pt, psi)
    assert abs(ov) ** 2 == pytest.approx(1 - eps, abs=1e-13)
    proj = np.sqrt(1 - eps) * pt * (ov / abs(ov))
    assert np.linalg.norm(psi - proj) ** 2 == pytest.approx(eps, rel=1e-9, abs=1e-15)
    # the truncated state has Schmidt rank chi across the cut and its Schmidt values are the
    # kept ones, renormalised
    st = np.linalg.svd(pt.reshape(2 ** (q + 1), -1), compute_uv=False)
    assert np.allclose(st[:chi], s[:chi] / np.sqrt(1 - eps), rtol=1e-10, atol=1e-13)
    assert np.all(st[chi:] < 1e-12)


def test_truncation_exact_when_chi_covers_the_cut():
    """eps = 0 (the a-posteriori estimate vanishes) whenever chi >= 2^(n/2): nothing is
    discarded and the step equals the untruncated one."""
    psi, pt, eps = _truncating_step(6, 2, 8, seed=44)
    assert eps < 1e-14
    assert 1 - abs(np.vdot(pt, psi)) ** 2 < 1e-13


def test_trajectory_average_matches_density_matrix():
    """Statistical agreement of 400 trajectories with the exact state (within 4 sigma
    per observable)."""
    c = I.brickwork(5, 4, seed=10, channel=I.depolarizing(0.2))
    zi_ex, zz_ex = dm.z_expectations(dm.run(c), 5)
    vals = []
    for t in range(400):
        m, _ = mps.trajectory(c, 8, t, 77)
        zi, zz = mps.z_expectations(m)
        vals.append(np.concatenate([zi, zz]))
    vals = np.array(vals)
    mean = vals.mean(0)
    se = vals.std(0, ddof=1) / np.sqrt(len(vals)) + 1e-12
    z = np.abs(mean - np.concatenate([zi_ex, zz_ex])) / se
    assert z.max() < 4.5


def test_born_sample_probabilities_are_the_born_rule():
    """The sampler's probability of each drawn bitstring (the product of its conditional
    probabilities) equals |<x|psi>|^2 of the dense state, and 20000 draws follow the Born
    distribution (chi^2 over the 64 outcomes)."""
    from oracle import mps as omps
    c = I.brickwork(6, 5, seed=61, channel=I.depolarizing(0.05))
    m, _ = omps.trajectory(c, 8, 3, 17)
    psi = m.to_vector()
    bits, probs = omps.born_sample(m, 20000, 99, 3)
    idx = (bits.astype(np.int64) * (1 << np.arange(5, -1, -1))).sum(1)   # qubit 0 most significant
    born = np.abs(psi) ** 2
    assert np.abs(probs - born[idx]).max() < 1e-12
    counts = np.bincount(idx, minlength=64)
    exp = born * len(idx)
    keep = exp > 5
    chi2 = float(((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum())
    assert chi2 < keep.sum() + 6 * np.sqrt(2 * keep.sum()), chi2


def test_born_samples_of_trajectories_follow_the_mixed_state():
    """Lemma on output distribution sampling: one Born sample from each of 3000 trajectories
    follows <x|rho|x> of the exact noisy state (orthogonal unravelling, 4 qubits)."""
    from oracle import mps as omps
    c = I.brickwork(4, 4, seed=62, channel=I.amplitude_damping(0.3))
    rho = dm.run(c)
    counts = np.zeros(16)
    T = 3000
    for t in range(T):
        m, _ = omps.trajectory(c, 4, t, 18, mode=0)
        b, _ = omps.born_sample(m, 1, 5, t)
        counts[int((b[0].astype(np.int64) * (1 << np.arange(3, -1, -1))).sum())] += 1
    exp = np.real(np.diag(rho)) * T
    keep = exp > 5
    chi2 = float(((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum())
    assert chi2 < keep.sum() + 6 * np.sqrt(2 * keep.sum()), chi2


def test_global_layering_without_truncation_equals_statevector():
    """(A state-independent unravelling: the optimal mixing is not unique, so rounding-level
    differences of the two representations could pick different optimal branches.)"""
    from oracle import mps as omps
    c = I.brickwork(6, 5, seed=63, channel=I.depolarizing(0.1))
    for t in range(4):
        m, eps = omps.trajectory_global(c, 8, t, 19, mode=0)
        psi = sv.trajectory(c, t, 19, mode=0)
        assert abs(abs(np.vdot(m.to_vector(), psi)) - 1.0) < 1e-12
        assert max(max(e) for e in eps) < 1e-14


def test_truncate_sweep_keeps_the_top_schmidt_values_of_the_first_cut():
    """The sweep's first bond sees the untruncated state: its kept values are the top-chi
    Schmidt values of the dense state at that cut, and its discarded weight their complement;
    afterwards every bond is at most chi and the state has norm 1."""
    from oracle import mps as omps
    c = I.brickwork(8, 6, seed=64, channel=I.depolarizing(0.02))
    m, _ = omps.trajectory(c, 16, 0, 20)
    psi = m.to_vector()
    s = np.linalg.svd(psi.reshape(2, -1), compute_uv=False)
    s2 = np.linalg.svd(psi.reshape(4, -1), compute_uv=False)
    eps = omps.truncate_sweep(m, 1)
    assert abs(eps[0] - s[1] ** 2 / np.sum(s ** 2)) < 1e-13
    assert max(m.bond_dims()) <= 1
    assert abs(np.linalg.norm(m.to_vector()) - 1.0) < 1e-13
    m2, _ = omps.trajectory(c, 16, 0, 20)
    eps2 = omps.truncate_sweep(m2, 3)
    assert eps2[0] == 0.0 or abs(eps2[0]) < 1e-15       # the first cut has rank <= 2
    assert abs(eps2[1] - np.sum(s2[3:] ** 2) / np.sum(s2 ** 2)) < 1e-12
