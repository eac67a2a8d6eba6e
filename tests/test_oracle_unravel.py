"""Pins of the oracle's locally entanglement-optimal unravelling (no GPU)."""
import math
import os

import numpy as np
import pytest

from oracle import unravel as U
from paper_2508_05745_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CHANNELS = {
    "dephasing": I.dephasing,
    "amplitude_damping": I.amplitude_damping,
    "depolarizing": I.depolarizing,
}


def _golden_choi():
    out = []
    for line in open(os.path.join(GOLD, "choi_closed_forms.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, r, e = line.split()
        out.append((name, float(r), float(e)))
    return out


@pytest.mark.parametrize("name,rate,eof", _golden_choi())
def test_choi_state_closed_forms(name, rate, eof):
    """Bell-state input (rho_q = I/2): EoF equals the paper's closed form and the returned
    decomposition reaches it with a complete Kraus set."""
    k = CHANNELS[name](rate)
    rho = np.eye(2) / 2
    out = U.optimal_mixing(rho, k)
    assert out["eof"] == pytest.approx(eof, abs=1e-12)
    kp = U.mixed_kraus(k, out["W"])
    p, eav = U.average_entanglement(rho, kp)
    assert eav == pytest.approx(eof, abs=1e-12)
    assert np.allclose(sum(x.conj().T @ x for x in kp), np.eye(2), atol=1e-13)
    assert p.sum() == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("p", [0.01, 0.2, 0.5])
def test_haar_optimal_fixed_mixings_reach_choi_eof(p):
    """The Haar-optimal (Hadamard) mixings of the appendix reach the Choi-state EoF with
    equal branch weights; checks the K'_j = sum_i U_ji K_i convention."""
    rho = np.eye(2) / 2
    h2 = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    for k, u in ((I.dephasing(p), h2), (I.amplitude_damping(p), h2),
                 (I.depolarizing(p), U.H4.real)):
        w = U.mixing(rho, k, U.MODE_FIXED, u)
        ps, eav = U.average_entanglement(rho, U.mixed_kraus(k, w))
        eof = U.optimal_mixing(rho, k)["eof"]
        assert eav == pytest.approx(eof, abs=1e-12)
        nz = ps[ps > 0]
        assert np.allclose(nz, 1.0 / len(nz))


@pytest.mark.parametrize("s,gamma", [(0.3, 0.1), (0.8, 0.5), (0.6, 0.9)])
def test_amplitude_damping_computational_schmidt_basis(s, gamma):
    """Remark in the appendix: C = 2 s sqrt(1-s^2) sqrt(1-gamma), attained by
    U = (1/sqrt2)[[1,-1],[1,1]]."""
    rho = np.diag([s * s, 1 - s * s]).astype(np.complex128)
    k = I.amplitude_damping(gamma)
    out = U.optimal_mixing(rho, k)
    c = 2 * s * math.sqrt(1 - s * s) * math.sqrt(1 - gamma)
    assert out["C"] == pytest.approx(c, abs=1e-12)
    u = np.array([[1, -1], [1, 1]]) / np.sqrt(2)
    _, eav = U.average_entanglement(rho, U.mixed_kraus(k, U.mixing(rho, k, U.MODE_FIXED, u)))
    assert eav == pytest.approx(out["eof"], abs=1e-12)


def test_bell_depolarizing_separability_threshold():
    """Bell state + depolarizing: C = max(0, 1 - 3p/2), separable from p = 2/3 on."""
    rho = np.eye(2) / 2
    for p in (0.1, 0.5, 0.66, 0.7, 0.9):
        out = U.optimal_mixing(rho, I.depolarizing(p))
        assert out["C"] == pytest.approx(max(0.0, 1 - 1.5 * p), abs=1e-12)
        assert out["separable"] == (p >= 2 / 3)
        _, eav = U.average_entanglement(rho, U.mixed_kraus(I.depolarizing(p), out["W"]))
        assert eav == pytest.approx(out["eof"], abs=1e-12)


def test_dephasing_worked_example_mixing_convention():
    """The worked dephasing example maps the mixed-unitary operators to the projective
    ones with K'_j = sum_i U_ji K_i."""
    p = 0.3
    rows = [l.split(";") for l in open(os.path.join(GOLD, "dephasing_projective_mixing.txt"))
            if not l.startswith("#")]
    u = np.zeros((3, 3))
    for r, c, e in rows:
        u[int(r), int(c)] = eval(e, {"sqrt": math.sqrt, "p": p})
    assert np.allclose(u @ u.T, np.eye(3), atol=1e-14)
    k = np.concatenate([I.dephasing(p), np.zeros((1, 2, 2))])
    kp = np.einsum("ji,iab->jab", u, k)
    want = [math.sqrt(1 - p) * np.eye(2), math.sqrt(p) * np.diag([1, 0]),
            math.sqrt(p) * np.diag([0, 1])]
    for a, b in zip(kp, want):
        assert np.allclose(a, b, atol=1e-14)


@pytest.mark.parametrize("chan", [I.depolarizing(0.02), I.amplitude_damping(0.3),
                                  I.dephasing(0.2), I.depolarizing(0.8),
                                  I.compose(I.amplitude_damping(0.05), I.dephasing(0.05))])
def test_random_states_reach_eof(chan):
    """On random single-qubit reduced states: E_av of the returned decomposition equals
    the Hill-Wootters EoF (via the Takagi lambdas) to 1e-12, the concurrence agrees with
    the independent sqrt(sqrt(rho) rho~ sqrt(rho)) route to 1e-7, the Kraus set is complete
    and z z^dag reproduces rho_eff."""
    for t in range(60):
        rho = I.random_density_matrices(1, t, rank=1 if t % 9 == 0 else 2)[0]
        out = U.optimal_mixing(rho, chan)
        kp = U.mixed_kraus(chan, out["W"])
        p, eav = U.average_entanglement(rho, kp)
        assert eav == pytest.approx(out["eof"], abs=1e-12)
        assert np.allclose(sum(x.conj().T @ x for x in kp), np.eye(2), atol=1e-12)
        reff = out["phi"] @ out["phi"].conj().T
        assert np.allclose(out["z"] @ out["z"].conj().T, reff, atol=1e-14)
        assert out["C"] == pytest.approx(U.concurrence_hill_wootters(reff), abs=1e-7)
        assert np.allclose(p, out["p"], atol=1e-14)


def test_brute_force_never_below_eof():
    """Random unitary mixings never beat the returned optimum."""
    rng = np.random.default_rng(5)
    chan = I.depolarizing(0.1)
    for t in range(5):
        rho = I.random_density_matrices(1, 100 + t)[0]
        eof = U.optimal_mixing(rho, chan)["eof"]
        for _ in range(400):
            u = I.haar_unitary(rng, 4)
            _, eav = U.average_entanglement(rho, U.mixed_kraus(chan, u.T))
            assert eav >= eof - 1e-12


def test_bell_depolarizing_u_theta_phi_grid_never_below_eof():
    """The U(theta, phi) family of the Bell + depolarizing example (two-parameter grid of
    mixings of the first two Paulis) never goes below EoF."""
    rho = np.eye(2) / 2
    chan = I.depolarizing(0.3)
    eof = U.optimal_mixing(rho, chan)["eof"]
    for th in np.linspace(0, np.pi, 13):
        for ph in np.linspace(0, 2 * np.pi, 13):
            u = np.eye(4, dtype=np.complex128)
            u[:2, :2] = [[np.cos(th), -np.exp(-1j * ph) * np.sin(th)],
                         [np.exp(1j * ph) * np.sin(th), np.cos(th)]]
            _, eav = U.average_entanglement(rho, U.mixed_kraus(chan, u.T))
            assert eav >= eof - 1e-12


def test_takagi_factorisation():
    rng = np.random.default_rng(2)
    for m in (2, 3, 4):
        a = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        tau = a + a.T
        sig, u = U.takagi(tau)
        assert np.allclose(u @ np.diag(sig) @ u.T, tau, atol=1e-12)
        assert np.allclose(u.conj().T @ u, np.eye(m), atol=1e-12)
        assert np.all(np.diff(sig) <= 1e-15)
    # rank-deficient symmetric matrix: null directions handled
    b = rng.standard_normal((3, 1)) + 1j * rng.standard_normal((3, 1))
    tau = b @ b.T
    sig, u = U.takagi(tau)
    assert np.allclose(u @ np.diag(sig) @ u.T, tau, atol=1e-12)
    assert np.allclose(u.conj().T @ u, np.eye(3), atol=1e-12)


def test_separable_angles_close_polygon():
    for lam in ([0.4, 0.3, 0.2, 0.1], [0.3, 0.3, 0.2, 0.2], [0.25] * 4, [0.5, 0.3, 0.2, 0.0],
                [0.4, 0.4, 0.1, 0.1], [0.35, 0.35, 0.0, 0.0]):
        th = U.separable_angles(np.array(lam))
        assert abs(np.sum(np.array(lam) * np.exp(2j * th))) < 1e-14
