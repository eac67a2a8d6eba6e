"""Certified error of truncated trajectory sampling (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The a-posteriori estimator of Thm. "Truncated Trajectory Sampling error" (Sec. "Upper bounds
on the simulation errors") from the truncations of the sampled trajectories, in the paper's
order:

* each approximation step (with local layering: one truncation of one bond after a gate)
  changes the trajectory state by a trace norm eps(step).  Two values are provided: the
  exact one for a single-bond truncation with renormalisation, 2 sqrt(eps_k) (the pure-state
  identity of the norms toolbox, ||psi psi^dag - phi phi^dag||_Tr = 2 sqrt(1 - |<psi|phi>|^2),
  with |<psi|phi>|^2 = 1 - eps_k for phi the renormalised projection), and the paper's
  computable bound 4 eps_trunc with eps_trunc = sqrt(2 sum_k eps_k) (Sec. "Errors based on
  MPS truncations", eq. MPS_truncation_error), one bond per step;
* the cumulated error of a trajectory is the sum over its steps (Prop. "systematic error",
  eq. cumulated_trajectory_error);
* capped at eps_max when it exceeds eps_max - 2 (Prop. "Path error bound"), 2 <= eps_max <= 2L;
* the estimator is the mean of the capped errors over the N sampled trajectories, and the
  systematic error is below it plus sqrt(eps_max^2 log(1/delta) / (2N)) with probability
  1 - delta (Prop. "systematic error bound", Hoeffding);
* concentration variants (Sec. "Improvements of the error bounds due to concentration"):
  layer l's errors weighted by alpha^(L-l), or for depolarizing noise of rate p by
  min(sqrt(8n) (1-p)^(L-l), 1), without the cap.

Also here: an exact enumeration of the Kraus tree *with* truncation (statevector, every
branch, the state projected onto its top-chi Schmidt vectors across the gate's cut after the
gate's noise), giving the exact truncated mixture sigma and the path-weighted cumulated
errors, for tiny circuits.

Pinned by: the exact per-step value against a brute-force trace norm; the paper's bound
above the exact value; eps = 0 without truncation; and, on enumerated trees, the exact
distance ||rho - sigma||_Tr (rho from the density-matrix oracle) below the path-weighted
bounds, capped and uncapped.
"""
from __future__ import annotations

import numpy as np

from . import sv as _sv
from . import unravel as _unr

STEP_EXACT = "exact"
STEP_PAPER = "paper"


def step_error(eps_k, kind: str = STEP_EXACT):
    """Trace-norm change of one single-bond truncation step with discarded weight eps_k."""
    e = np.maximum(np.asarray(eps_k, dtype=np.float64), 0.0)
    if kind == STEP_EXACT:
        return 2.0 * np.sqrt(e)
    if kind == STEP_PAPER:
        return 4.0 * np.sqrt(2.0 * e)
    raise ValueError(kind)


def layer_weights(n_layers: int, scheme: str = "none", alpha: float = 1.0, p: float = 0.0, n: int = 1):
    """Weight of layer l = 0..L-1's errors: 1 (Thm. 1), alpha^(L-1-l), or for depolarizing
    noise min(sqrt(8n) (1-p)^(L-1-l), 1) (layers counted from 1 in the paper: L - l)."""
    L = n_layers
    k = np.arange(L)
    if scheme == "none":
        return np.ones(L)
    if scheme == "alpha":
        return alpha ** (L - 1 - k).astype(np.float64)
    if scheme == "depolarizing":
        return np.minimum(np.sqrt(8.0 * n) * (1.0 - p) ** (L - 1 - k).astype(np.float64), 1.0)
    raise ValueError(scheme)


def trajectory_error(eps_by_layer, kind: str = STEP_EXACT, weights=None) -> float:
    """Cumulated error of one trajectory: sum over layers of weight * sum of its steps'
    errors (eps_by_layer: one sequence of discarded weights per layer)."""
    tot = 0.0
    for l, eps in enumerate(eps_by_layer):
        w = 1.0 if weights is None else float(weights[l])
        tot += w * float(np.sum(step_error(eps, kind)))
    return tot


def capped(eps_tot, eps_max: float):
    """eps_bound of Prop. "Path error bound": eps_tot if eps_tot <= eps_max - 2, else eps_max."""
    e = np.asarray(eps_tot, dtype=np.float64)
    return np.where(e <= eps_max - 2.0, e, eps_max)


def estimate(eps_tots, eps_max: float = 4.0, delta: float = 0.05):
    """(eps_hat, buffer, bound): the mean capped error of the sampled trajectories, the
    Hoeffding buffer sqrt(eps_max^2 log(1/delta) / (2N)), and their sum."""
    e = capped(eps_tots, eps_max)
    n = e.size
    hat = float(np.mean(e))
    buf = float(np.sqrt(eps_max ** 2 * np.log(1.0 / delta) / (2.0 * n)))
    return hat, buf, hat + buf


def truncate_cut(psi: np.ndarray, n: int, q: int, chi: int):
    """Project a normalised state onto its chi largest Schmidt vectors across the cut
    (0..q | q+1..n-1), renormalise; returns (state, discarded weight)."""
    m = psi.reshape(2 ** (q + 1), -1)
    u, s, vh = np.linalg.svd(m, full_matrices=False)
    d = min(chi, s.size)
    tot = float(np.sum(s ** 2))
    kept = float(np.sum(s[:d] ** 2))
    out = (u[:, :d] * s[:d]) @ vh[:d]
    return out.reshape(-1) / np.sqrt(kept), (tot - kept) / tot


def truncated_tree(circuit, chi: int, mode=_unr.MODE_OPTIMAL, fixed_u=None):
    """All paths of the Kraus tree with a truncation to chi after every gate (its noise
    included, local layering): returns (sigma, [(probability, per-layer discarded-weight
    lists) per leaf])."""
    n = circuit.n
    psi0 = np.zeros(2 ** n, dtype=np.complex128)
    psi0[0] = 1.0
    ops = []
    for l in range(circuit.depth):
        for kind, q in _sv.sweep_ops(circuit, l):
            if kind == "gate":
                ops.append(("gate", l, q))
            for x in _sv.event_qubits(circuit, l, kind, q):
                ops.append(("noise", l, x))
            if kind == "gate":
                ops.append(("trunc", l, q))
    sigma = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    leaves = []
    stack = [(psi0, 1.0, 0, [[] for _ in range(circuit.depth)])]
    while stack:
        psi, w, i, eps = stack.pop()
        while i < len(ops) and ops[i][0] != "noise":
            kind, l, q = ops[i]
            if kind == "gate":
                psi = _sv.apply_two(psi, n, q, circuit.gate(l, q))
            else:
                psi, e = truncate_cut(psi, n, q, chi)
                eps = [list(x) for x in eps]
                eps[l].append(e)
            i += 1
        if i == len(ops):
            sigma += w * np.outer(psi, psi.conj())
            leaves.append((w, eps))
            continue
        _, l, x = ops[i]
        kraus = circuit.kraus(int(circuit.events[l, x]))
        rho_q = _sv.reduced_one(psi, n, x)
        rho_q = rho_q / np.trace(rho_q).real
        kp = _unr.mixed_kraus(kraus, _unr.mixing(rho_q, kraus, mode, fixed_u))
        for k in kp:
            out = _sv.apply_one(psi, n, x, k)
            pj = float(np.vdot(out, out).real)
            if pj > 1e-300:
                stack.append((out / np.sqrt(pj), w * pj, i + 1, eps))
    return sigma, leaves


def trace_norm(a: np.ndarray) -> float:
    """Trace norm of a Hermitian matrix: the sum of |eigenvalues|."""
    return float(np.sum(np.abs(np.linalg.eigvalsh(a))))
