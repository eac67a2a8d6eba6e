"""Statevector trajectories (oracle, tiny widths).

One trajectory of the Kraus tree (Sec. "Class of Truncated Trajectory Sampling Algorithms")
with the channel-unravelling subprocedure (Alg. 1) applied to every noise event and no
approximation: after a gate, each noise event on qubit q

  * forms the reduced state rho_q of the current |psi>,
  * chooses the Kraus mixing W (unravelling mode),
  * computes p_j = ||K'_j psi||^2 (Eq. Kraus_to_ensemble),
  * draws u from the counter-based generator keyed by (trajectory, layer, qubit) and picks
    branch j,
  * sets psi <- K'_j psi / sqrt(p_j).

Event order (pinned reading; it only matters once truncation is involved but is kept
identical everywhere): layer l is swept left to right when l is even and right to left
when l is odd; each gate is followed by the noise on its lower qubit, then on its upper
qubit; noise on a qubit left idle by the layer is applied when the sweep reaches it.

Pinned by: the exact Kraus-tree average, the density-matrix oracle within statistical
error, and norm 1 after every event.
"""
from __future__ import annotations

import numpy as np

from . import rng as _rng
from . import unravel as _unr


def sweep_ops(circuit, layer: int):
    """Ordered operations of one layer: ('gate', q) for the pair (q, q+1) and ('idle', q)
    for noise on a qubit not touched by a gate in this layer."""
    n = circuit.n
    pairs = circuit.pairs(layer)
    covered = set()
    for q in pairs:
        covered.update((q, q + 1))
    ops = [(q, "gate") for q in pairs]
    ops += [(q, "idle") for q in range(n) if q not in covered and circuit.events[layer, q] >= 0]
    ops.sort(key=lambda t: t[0])
    if layer % 2 == 1:
        ops.reverse()
    return [(kind, q) for q, kind in ops]


def event_qubits(circuit, layer: int, kind: str, q: int):
    qs = [q, q + 1] if kind == "gate" else [q]
    return [x for x in qs if circuit.events[layer, x] >= 0]


def reduced_one(psi: np.ndarray, n: int, q: int) -> np.ndarray:
    t = np.moveaxis(psi.reshape((2,) * n), q, 0).reshape(2, -1)
    return t @ t.conj().T


def apply_one(psi: np.ndarray, n: int, q: int, k: np.ndarray) -> np.ndarray:
    t = np.tensordot(k, psi.reshape((2,) * n), axes=([1], [q]))
    return np.moveaxis(t, 0, q).reshape(-1)


def apply_two(psi: np.ndarray, n: int, q: int, g: np.ndarray) -> np.ndarray:
    t = np.tensordot(g.reshape(2, 2, 2, 2), psi.reshape((2,) * n), axes=([2, 3], [q, q + 1]))
    return np.moveaxis(t, [0, 1], [q, q + 1]).reshape(-1)


def choose_mixing(rho_q, kraus, mode, fixed_u, replay):
    """W from the unravelling mode, or the next recorded W of a replay (checked)."""
    if replay is not None:
        return replay.next(rho_q, kraus)
    return _unr.mixing(rho_q, kraus, mode, fixed_u)


class Replay:
    """Follows a recorded sequence of mixings W (e.g. the ones a GPU run chose) and checks
    each one: the induced Kraus set must be complete and, for the optimal mode, its average
    entanglement must equal the entanglement of formation of this side's own reduced state
    (any optimal decomposition is acceptable; the optimum is not unique)."""

    def __init__(self, ws, check_optimal=True):
        self.ws = list(ws)
        self.i = 0
        self.check_optimal = check_optimal
        self.max_gap = 0.0
        self.max_incomplete = 0.0

    def next(self, rho_q, kraus):
        w = np.asarray(self.ws[self.i], dtype=np.complex128)[: kraus.shape[0]]
        self.i += 1
        kp = _unr.mixed_kraus(kraus, w)
        inc = np.abs(sum(k.conj().T @ k for k in kp) - np.eye(2)).max()
        self.max_incomplete = max(self.max_incomplete, float(inc))
        if self.check_optimal:
            _, eav = _unr.average_entanglement(rho_q, kp)
            eof = _unr.optimal_mixing(rho_q, kraus)["eof"]
            self.max_gap = max(self.max_gap, abs(eav - eof))
        return w


def noise_event(psi, n, q, kraus, mode, u, fixed_u=None, record=None, replay=None):
    rho_q = reduced_one(psi, n, q)
    rho_q = rho_q / np.trace(rho_q).real
    w = choose_mixing(rho_q, kraus, mode, fixed_u, replay)
    kp = _unr.mixed_kraus(kraus, w)
    outs = [apply_one(psi, n, q, k) for k in kp]
    p = np.array([np.vdot(o, o).real for o in outs])
    j = _rng.sample_branch(p, u)
    if record is not None:
        record.append(dict(q=q, p=p, j=j, W=w))
    return outs[j] / np.sqrt(p[j])


def trajectory(circuit, traj: int, seed: int, mode: int = _unr.MODE_OPTIMAL, fixed_u=None,
               layers=None, record=None, replay=None) -> np.ndarray:
    n = circuit.n
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    for l in range(circuit.depth if layers is None else layers):
        for kind, q in sweep_ops(circuit, l):
            if kind == "gate":
                psi = apply_two(psi, n, q, circuit.gate(l, q))
            for x in event_qubits(circuit, l, kind, q):
                ch = int(circuit.events[l, x])
                u = _rng.uniform(seed, traj, l, x)
                psi = noise_event(psi, n, x, circuit.kraus(ch), mode, u, fixed_u, record, replay)
    return psi


def z_expectations(psi: np.ndarray, n: int):
    prob = (np.abs(psi) ** 2).reshape((2,) * n)
    zi, zz = [], []
    for i in range(n):
        p = prob.sum(axis=tuple(a for a in range(n) if a != i))
        zi.append(p[0] - p[1])
    for i in range(n - 1):
        p = prob.sum(axis=tuple(a for a in range(n) if a not in (i, i + 1)))
        zz.append(p[0, 0] - p[0, 1] - p[1, 0] + p[1, 1])
    return np.array(zi), np.array(zz)
