"""Exact enumeration of the Kraus tree (oracle, tiny circuits).

Every path from the root to a leaf of the Kraus tree (Sec. "Class of Truncated Trajectory
Sampling Algorithms", Fig. kraus_tree) is followed with its probability: at each noise
event the unravelling is chosen from the current branch state (adaptive) and every branch
j with p_j > 0 is expanded.  Without approximation the probability-weighted average of the
leaf states is the exact noisy state, whatever the unravelling.

Pinned against the density-matrix oracle (an independent computation).
"""
from __future__ import annotations

import numpy as np

from . import sv as _sv
from . import unravel as _unr


def average_state(circuit, mode=_unr.MODE_OPTIMAL, fixed_u=None, layers=None):
    n = circuit.n
    psi0 = np.zeros(2 ** n, dtype=np.complex128)
    psi0[0] = 1.0
    ops = []
    for l in range(circuit.depth if layers is None else layers):
        for kind, q in _sv.sweep_ops(circuit, l):
            if kind == "gate":
                ops.append(("gate", l, q))
            for x in _sv.event_qubits(circuit, l, kind, q):
                ops.append(("noise", l, x))

    rho = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    stack = [(psi0, 1.0, 0)]
    while stack:
        psi, w, i = stack.pop()
        while i < len(ops) and ops[i][0] == "gate":
            _, l, q = ops[i]
            psi = _sv.apply_two(psi, n, q, circuit.gate(l, q))
            i += 1
        if i == len(ops):
            rho += w * np.outer(psi, psi.conj())
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
                stack.append((out / np.sqrt(pj), w * pj, i + 1))
    return rho
