"""Pins of the certified error estimator (Thm. "Truncated Trajectory Sampling error" and its
propositions) in the oracle: per-step values against brute-force trace norms, and the bound
against the exact distance between the exact noisy state and the exact truncated mixture on
enumerated Kraus trees (no GPU)."""
import numpy as np
import pytest

from oracle import dm
from oracle import error as E
from oracle import unravel as U
from paper_2508_05745_amd import inputs as I


def test_step_error_exact_is_the_trace_norm_of_one_truncation():
    """2 sqrt(eps_k) equals ||psi psi^dag - phi phi^dag||_Tr computed from the eigenvalues of
    the difference, for random states truncated at random cuts; the paper's bound
    4 sqrt(2 eps_k) lies above it."""
    rng = np.random.default_rng(3)
    for n, q, chi in [(6, 2, 2), (7, 3, 3), (8, 3, 5), (5, 1, 1)]:
        psi = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
        psi /= np.linalg.norm(psi)
        phi, eps = E.truncate_cut(psi, n, q, chi)
        d = E.trace_norm(np.outer(psi, psi.conj()) - np.outer(phi, phi.conj()))
        assert eps > 1e-3
        assert E.step_error(eps, E.STEP_EXACT) == pytest.approx(d, rel=1e-10)
        assert E.step_error(eps, E.STEP_PAPER) >= d


def test_no_truncation_no_error():
    """chi >= 2^(n/2): every discarded weight and the estimate vanish."""
    c = I.brickwork(4, 2, seed=5, channel=I.depolarizing(0.1))
    sigma, leaves = E.truncated_tree(c, 4)
    assert np.abs(sigma - dm.run(c)).max() < 1e-12
    tots = [E.trajectory_error(eps) for _, eps in leaves]
    assert max(tots) < 1e-6        # 2 sqrt(eps) of rounding-level eps
    assert E.estimate(np.zeros(10), 4.0, 0.05)[0] == 0.0


@pytest.mark.parametrize("mode,chi,seed,ch", [(U.MODE_OPTIMAL, 1, 7, "dep"), (U.MODE_ORTHOGONAL, 1, 8, "dep"),
                                              (U.MODE_OPTIMAL, 1, 9, "ad"), (U.MODE_OPTIMAL, 2, 10, "deph")])
def test_bound_dominates_the_exact_systematic_error(mode, chi, seed, ch):
    """Prop. "systematic error" and "Path error bound": the exact trace distance between the
    exact noisy state (density-matrix oracle) and the exact truncated mixture (all branches
    enumerated) is at most the path-weighted cumulated error, with the exact per-step values
    and the paper's bounds, and with the eps_max cap (eps_max = 2 and 4)."""
    chan = {"dep": I.depolarizing(0.15), "ad": I.amplitude_damping(0.3), "deph": I.dephasing(0.3)}[ch]
    n, depth = 4, 2
    c = I.brickwork(n, depth, seed=seed, channel=chan)
    sigma, leaves = E.truncated_tree(c, chi, mode)
    rho = dm.run(c)
    dist = E.trace_norm(rho - sigma)
    assert abs(np.trace(sigma).real - 1) < 1e-12
    assert dist > 1e-3                       # the truncation matters
    for kind in (E.STEP_EXACT, E.STEP_PAPER):
        tots = np.array([E.trajectory_error(eps, kind) for _, eps in leaves])
        w = np.array([p for p, _ in leaves])
        assert dist <= float(np.dot(w, tots)) + 1e-12
        for eps_max in (2.0, 4.0):
            assert dist <= float(np.dot(w, E.capped(tots, eps_max))) + 1e-12


def test_capping_rule():
    e = np.array([0.0, 0.5, 1.99, 2.0, 2.01, 7.0])
    assert np.array_equal(E.capped(e, 4.0), [0.0, 0.5, 1.99, 2.0, 4.0, 4.0])
    assert np.array_equal(E.capped(e, 2.0), [0.0, 2.0, 2.0, 2.0, 2.0, 2.0])


def test_hoeffding_buffer_covers_the_mean():
    """The buffer sqrt(eps_max^2 log(1/delta) / (2N)) of a mean of N variables in [0, eps_max]:
    over many repetitions with the mean known, the true mean exceeds the estimate plus the
    buffer in at most a delta fraction (Hoeffding's inequality; here well below)."""
    rng = np.random.default_rng(11)
    eps_max, delta, n = 4.0, 0.1, 50
    true_mean = 0.25 * eps_max * 0.6   # Beta(1.5, 2.5)-distributed values scaled to [0, eps_max]
    fails = 0
    for _ in range(2000):
        x = eps_max * rng.beta(1.5, 2.5, size=n)
        hat, buf, bound = E.estimate(x, eps_max, delta)
        assert buf == pytest.approx(np.sqrt(eps_max ** 2 * np.log(1 / delta) / (2 * n)))
        fails += true_mean > bound
    assert fails / 2000 <= delta


def test_concentration_weights():
    """alpha = 1 and p = 0 reduce the concentration variants to the plain sum (the
    depolarizing weight is capped at 1); the weights decay towards early layers."""
    assert np.array_equal(E.layer_weights(5, "alpha", alpha=1.0), np.ones(5))
    assert np.array_equal(E.layer_weights(5, "depolarizing", p=0.0, n=10), np.ones(5))
    w = E.layer_weights(200, "depolarizing", p=0.02, n=100)
    assert w[-1] == 1.0 and np.all(np.diff(w) >= 0) and w[0] < 1.0
    assert w[0] == pytest.approx(np.sqrt(800) * 0.98 ** 199)
