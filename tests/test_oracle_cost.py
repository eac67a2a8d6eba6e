"""Pins of the unravelling cost and its reference gradient (no GPU)."""
import numpy as np
import pytest

from oracle import cost as CO
from oracle import unravel as U
from paper_2508_05745_amd import inputs as I


def _u_opt(rho, k):
    w = U.optimal_mixing(rho, k)["W"]
    u = np.zeros((4, 4), dtype=np.complex128)
    u[:, : w.shape[0]] = w.T  # K'_j = sum_i U_ji K_i  <=>  U = W^T (zero columns past r)
    return u


def test_generators_are_a_hermitian_basis():
    g = CO.generators()
    assert np.allclose(g, np.conj(np.transpose(g, (0, 2, 1))))
    m = g.reshape(16, 16)
    assert np.linalg.matrix_rank(np.concatenate([m.real, m.imag], axis=1)) == 16


@pytest.mark.parametrize("seed", range(6))
def test_linear_cost_minimum_is_half_concurrence_squared(seed):
    """At the Wootters mixing every branch has concurrence C, so f_lin = C^2 / 2; any other
    mixing costs at least that (convexity of c^2/2 and sum_j p_j c_j >= C)."""
    k = I.depolarizing(0.02 + 0.05 * seed)
    rho = I.random_density_matrices(1, 40 + seed)[0]
    out = U.optimal_mixing(rho, k)
    uo = _u_opt(rho, k)
    f = CO.cost(rho, k, uo, CO.KIND_LINEAR)
    assert f == pytest.approx(out["C"] ** 2 / 2, abs=1e-12)
    rng = np.random.default_rng(seed)
    for _ in range(50):
        assert CO.cost(rho, k, I.haar_unitary(rng, 4), CO.KIND_LINEAR) >= f - 1e-12


@pytest.mark.parametrize("kind", [CO.KIND_LINEAR, CO.KIND_RENYI2])
def test_gradient_vanishes_at_optimum(kind):
    k = I.depolarizing(0.02)
    rho = I.random_density_matrices(1, 7)[0]
    uo = _u_opt(rho, k)
    f, g = CO.grad_torch(rho, k, np.zeros(16), uo, kind)
    assert np.abs(g).max() < 1e-8
    assert np.abs(CO.grad_fd(rho, k, np.zeros(16), uo, kind)).max() < 1e-7


@pytest.mark.parametrize("kind", [CO.KIND_LINEAR, CO.KIND_RENYI2])
def test_autograd_matches_finite_differences(kind):
    rng = np.random.default_rng(3)
    k = I.depolarizing(0.02)
    for t in range(4):
        rho = I.random_density_matrices(1, 60 + t)[0]
        params = rng.normal(0, 0.1, 16)
        uref = I.haar_unitary(rng, 4)
        f, g = CO.grad_torch(rho, k, params, uref, kind)
        assert f == pytest.approx(CO.cost_params(rho, k, params, uref, kind), abs=1e-13)
        gfd = CO.grad_fd(rho, k, params, uref, kind)
        assert np.linalg.norm(g - gfd) <= 1e-6 * np.linalg.norm(g) + 1e-8


def test_rho_from_theta_is_reduced_state():
    th = I.random_two_site_states(3, 4, 5, seed=1, dtype=np.complex128)
    for t in th:
        r = CO.rho_from_theta(t)
        psi = t.transpose(1, 0, 2, 3).reshape(2, -1)      # target index first
        assert np.allclose(r, psi @ psi.conj().T, atol=1e-15)
        assert abs(np.trace(r) - 1) < 1e-14


@pytest.mark.parametrize("seed", range(6))
def test_renyi2_cost_at_optimum_closed_form(seed):
    """Every branch of Wootters' decomposition is a pure two-qubit state of concurrence C
    (appendix on Wootters' optimal decomposition), whose target purity is 1 - C^2/2; so the
    Renyi-2 cost at the optimal mixing is -log2(1 - C^2/2) (base-2 logarithm), and, the
    function -log2(1 - c^2/2) being convex and increasing in c, no Haar-random mixing does
    better."""
    k = [I.depolarizing(0.03 + 0.04 * seed), I.amplitude_damping(0.1 + 0.1 * seed),
         I.dephasing(0.05 + 0.1 * seed)][seed % 3]
    rho = I.random_density_matrices(1, 80 + seed)[0]
    out = U.optimal_mixing(rho, k)
    c = out["C"]
    assert c > 1e-3
    f = CO.cost(rho, k, _u_opt(rho, k), CO.KIND_RENYI2)
    assert f == pytest.approx(-np.log2(1 - c * c / 2), rel=1e-11, abs=1e-13)
    rng = np.random.default_rng(100 + seed)
    for _ in range(50):
        assert CO.cost(rho, k, I.haar_unitary(rng, 4), CO.KIND_RENYI2) >= f - 1e-12


def test_renyi2_cost_special_values():
    """Closed values: the identity channel on the maximally mixed qubit leaves one branch
    of target purity 1/2, so f_R2 = -log2(1/2) = 1 bit and f_lin = 1/2; a pure target state
    gives pure branches (f = 0) for any mixing."""
    k = np.eye(2, dtype=np.complex128)[None]
    rho = np.eye(2, dtype=np.complex128) / 2
    u = np.eye(4, dtype=np.complex128)
    assert CO.cost(rho, k, u, CO.KIND_RENYI2) == pytest.approx(1.0, abs=1e-15)
    assert CO.cost(rho, k, u, CO.KIND_LINEAR) == pytest.approx(0.5, abs=1e-15)
    pure = np.array([[0.36, 0.48], [0.48, 0.64]], dtype=np.complex128)
    rng = np.random.default_rng(5)
    for kk in (I.depolarizing(0.2), I.amplitude_damping(0.3)):
        for _ in range(5):
            uu = I.haar_unitary(rng, 4)
            assert abs(CO.cost(pure, kk, uu, CO.KIND_RENYI2)) < 1e-13
            assert abs(CO.cost(pure, kk, uu, CO.KIND_LINEAR)) < 1e-13


@pytest.mark.parametrize("kind", [0, 1])
def test_bond_cost_equals_qubit_cost_for_two_qubits(kind):
    """With chi_L = chi_R = 1 the block is two qubits, its internal bond separates the noisy
    qubit from the rest of the block, and the internal-bond cost equals the noisy-qubit cost."""
    rng = np.random.default_rng(31 + kind)
    for _ in range(10):
        th = I.random_two_site_states(1, 1, 1, seed=int(rng.integers(1 << 30)), dtype=np.complex128)[0]
        k = I.depolarizing(0.2) if _ % 2 else I.amplitude_damping(0.3)
        u = I.haar_unitaries(1, seed=int(rng.integers(1 << 30)))[0]
        rho = CO.rho_from_theta(th)
        assert abs(CO.bond_cost(th, k, u, kind) - CO.cost(rho / np.trace(rho).real, k, u, kind)) < 1e-13


@pytest.mark.parametrize("kind", [0, 1])
def test_bond_cost_gradient_finite_differences(kind):
    rng = np.random.default_rng(41 + kind)
    th = I.random_two_site_states(1, 3, 4, seed=5, dtype=np.complex128)[0]
    k = I.depolarizing(0.1)
    for _ in range(3):
        params = rng.normal(0, 0.3, 16)
        u_ref = I.haar_unitaries(1, seed=int(rng.integers(1 << 30)))[0]
        f, g = CO.bond_grad_torch(th, k, params, u_ref, kind)
        assert abs(f - CO.bond_cost_params(th, k, params, u_ref, kind)) < 1e-13
        gfd = CO.bond_grad_fd(th, k, params, u_ref, kind)
        assert np.linalg.norm(g - gfd) < 1e-7 * max(1.0, np.linalg.norm(g))


def test_bond_cost_of_a_product_block_is_the_qubit_cost_of_its_left_part():
    """theta = phi (x) chi with phi on (a, s) and chi on (t, b): every branch stays a product
    across the internal bond after noise on s, so the bond's entanglement is that of (a : s)
    inside phi; with chi_L = 1 (phi a single qubit) that is zero for every mixing."""
    rng = np.random.default_rng(7)
    phi = rng.standard_normal((1, 2)) + 1j * rng.standard_normal((1, 2))
    chi = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    th = np.einsum("as,tb->astb", phi, chi)
    u = I.haar_unitaries(1, seed=3)[0]
    for kind in (0, 1):
        assert abs(CO.bond_cost(th, I.depolarizing(0.3), u, kind)) < 1e-14
