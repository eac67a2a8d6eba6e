"""Pins of the Lindbladian oracle (no GPU): the two remarks of the appendix on typical jump
operators, trace preservation of the Choi-derived Kraus sets, and first-order convergence of
the Trotterised density matrix to the exact exp(L t)."""
import math

import numpy as np
import pytest

from oracle import dm as odm
from oracle import lindblad as OL
from paper_2508_05745_amd import inputs as I

P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)       # |0><0|
SM = np.array([[0, 1], [0, 0]], dtype=np.complex128)       # |0><1|


def _superop(kraus):
    return sum(np.kron(k, k.conj()) for k in kraus)


def _same_up_to_phase(a, b, tol):
    i = np.unravel_index(np.argmax(np.abs(b)), b.shape)
    ph = a[i] / b[i]
    return abs(abs(ph) - 1.0) < tol and np.abs(a - ph * b).max() < tol


@pytest.mark.parametrize("gamma,dt", [(0.1, 0.01), (1.0, 0.2), (3.0, 0.5)])
def test_dephasing_jump_gives_the_dephasing_channel(gamma, dt):
    """c = |0><0|: a dephasing channel of rate p = 1 - exp(-gamma dt / 2), decomposed into the
    rescaled identity and Z (appendix, first remark on typical jump operators)."""
    k = OL.jump_kraus([(P0, gamma)], dt)
    p = 1.0 - math.exp(-gamma * dt / 2)
    assert k.shape[0] == 2
    assert np.abs(_superop(k) - _superop(I.dephasing(p))).max() < 1e-14
    assert _same_up_to_phase(k[0], math.sqrt(1 - p / 2) * np.eye(2), 1e-12)
    assert _same_up_to_phase(k[1], math.sqrt(p / 2) * np.diag([1.0, -1.0]), 1e-12)


@pytest.mark.parametrize("gamma,dt", [(0.1, 0.01), (1.0, 0.2), (3.0, 0.5)])
def test_lowering_jump_gives_amplitude_damping(gamma, dt):
    """c = |0><1|: amplitude damping of rate gamma_AD = 1 - exp(-gamma dt), in its usual two
    operators (appendix, second remark)."""
    k = OL.jump_kraus([(SM, gamma)], dt)
    g = 1.0 - math.exp(-gamma * dt)
    assert k.shape[0] == 2
    assert np.abs(_superop(k) - _superop(I.amplitude_damping(g))).max() < 1e-14
    assert _same_up_to_phase(k[0], np.diag([1.0, math.sqrt(1 - g)]), 1e-12)
    assert _same_up_to_phase(k[1], math.sqrt(g) * SM, 1e-12)


def test_random_jumps_give_orthogonal_trace_preserving_kraus_sets():
    rng = np.random.default_rng(5)
    for _ in range(20):
        jumps = [(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)), rng.uniform(0.1, 2.0))
                 for _ in range(rng.integers(1, 3))]
        k = OL.jump_kraus(jumps, rng.uniform(0.01, 0.5))
        assert 1 <= k.shape[0] <= 4
        assert np.abs(sum(x.conj().T @ x for x in k) - np.eye(2)).max() < 1e-13
        g = np.array([[np.vdot(a, b) for b in k] for a in k])
        assert np.abs(g - np.diag(np.diag(g))).max() < 1e-13       # orthogonal operators


def test_pair_terms_sum_to_the_hamiltonian():
    m = I.lindblad_heisenberg(n=4, steps=1)
    X, Y, Z = (np.array(a, dtype=np.complex128) for a in ([[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]))
    def site(op, q):
        return np.kron(np.kron(np.eye(2 ** q), op), np.eye(2 ** (4 - q - 1)))
    h = sum(site(Y, q) @ site(Y, q + 1) for q in range(3)) + sum(site(0.35 * X + 0.35 * Y + 0.5 * Z, q) for q in range(4))
    hp = sum(np.kron(np.kron(np.eye(2 ** q), m.pair_hamiltonian(q)), np.eye(2 ** (4 - q - 2))) for q in range(3))
    assert np.abs(h - hp).max() < 1e-14


@pytest.mark.parametrize("kind", ["heisenberg", "random"])
def test_trotterised_density_matrix_converges_to_exp_lt(kind):
    """Fixed t = 0.4 on 4 qubits: the Trotter error of the circuit's exact density matrix
    halves with the time step (first order) and is small."""
    def model(steps):
        dt = 0.4 / steps
        if kind == "heisenberg":
            return I.lindblad_heisenberg(n=4, steps=steps, dt=dt, gamma_ad=1.0 - math.exp(-0.5 * dt))
        return I.lindblad_random_ti(n=4, steps=steps, dt=dt, gamma_ad=1.0 - math.exp(-0.5 * dt), seed=3)
    errs = []
    for steps in (8, 16, 32):
        m = model(steps)
        assert abs(m.jumps[0][1] - 1.0) < 1e-12          # the same jump rate gamma = 1 for every dt
        exact = OL.exact_state(m, 0.4)
        rho = OL.trotter_state(m)
        assert abs(np.trace(rho) - 1.0) < 1e-13
        errs.append(np.abs(rho - exact).sum())
    r1, r2 = errs[1] / errs[0], errs[2] / errs[1]
    assert errs[2] < 0.2 and 0.45 < r1 < 0.55 and 0.45 < r2 < 0.55, errs


def test_lindblad_circuit_layout():
    m = I.lindblad_heisenberg(n=5, steps=2)
    c = OL.circuit(m)
    assert c.depth == 4 and (c.events == 0).all() and c.n_kraus[0] == 2
    for l in range(c.depth):
        for q in c.pairs(l):
            assert np.abs(c.gate(l, q) - OL.trotter_gate(m.pair_hamiltonian(q), m.dt)).max() == 0.0
    # a circuit's density matrix is a state
    rho = odm.run(c)
    assert abs(np.trace(rho) - 1) < 1e-13 and np.linalg.eigvalsh(0.5 * (rho + rho.conj().T)).min() > -1e-13
