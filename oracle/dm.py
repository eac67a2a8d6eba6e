"""Exact density-matrix evolution of a noisy brickwork circuit (oracle, tiny widths).

rho^(L) is the composition of every layer's channel applied to |0..0><0..0| (the exact
state of the Kraus tree without approximation, Sec. "Class of Truncated Trajectory
Sampling Algorithms" and the state notation of the error-bound appendix): each gate is
rho -> G rho G^dag on its pair, each noise event rho -> sum_i K_i rho K_i^dag on its qubit.
Within a layer the channels act on disjoint qubits, so their order does not matter.

Pinned by: trace 1 and Hermitian PSD output, hand-computed two-qubit cases, and the
statevector / Kraus-tree enumerations that must average to it.
"""
from __future__ import annotations

import numpy as np


def _apply_two(rho: np.ndarray, n: int, q: int, g: np.ndarray) -> np.ndarray:
    """G on qubits (q, q+1) from the left and G^dag from the right; rho is (2,)*2n."""
    g4 = g.reshape(2, 2, 2, 2)
    rho = np.tensordot(g4, rho, axes=([2, 3], [q, q + 1]))          # new axes first
    rho = np.moveaxis(rho, [0, 1], [q, q + 1])
    rho = np.tensordot(rho, g4.conj(), axes=([n + q, n + q + 1], [2, 3]))
    return np.moveaxis(rho, [2 * n - 2, 2 * n - 1], [n + q, n + q + 1])


def _apply_one(rho: np.ndarray, n: int, q: int, k: np.ndarray) -> np.ndarray:
    rho = np.moveaxis(np.tensordot(k, rho, axes=([1], [q])), 0, q)
    rho = np.tensordot(rho, k.conj(), axes=([n + q], [1]))
    return np.moveaxis(rho, 2 * n - 1, n + q)


def initial(n: int) -> np.ndarray:
    rho = np.zeros((2,) * (2 * n), dtype=np.complex128)
    rho[(0,) * (2 * n)] = 1.0
    return rho


def apply_channel(rho: np.ndarray, n: int, q: int, kraus: np.ndarray) -> np.ndarray:
    out = np.zeros_like(rho)
    for k in kraus:
        out += _apply_one(rho, n, q, k)
    return out


def run(circuit, layers=None) -> np.ndarray:
    """Exact final state as a 2^n x 2^n matrix."""
    n = circuit.n
    rho = initial(n)
    for l in range(circuit.depth if layers is None else layers):
        for q in circuit.pairs(l):
            rho = _apply_two(rho, n, q, circuit.gate(l, q))
        for q in range(n):
            ch = int(circuit.events[l, q])
            if ch >= 0:
                rho = apply_channel(rho, n, q, circuit.kraus(ch))
    return rho.reshape(2 ** n, 2 ** n)


def z_expectations(rho: np.ndarray, n: int):
    """<Z_i> (n values) and <Z_i Z_{i+1}> (n-1 values) of a 2^n x 2^n density matrix."""
    diag = np.real(np.diag(rho)).reshape((2,) * n)
    zi, zz = [], []
    for i in range(n):
        p = diag.sum(axis=tuple(a for a in range(n) if a != i))
        zi.append(p[0] - p[1])
    for i in range(n - 1):
        p = diag.sum(axis=tuple(a for a in range(n) if a not in (i, i + 1)))
        zz.append(p[0, 0] - p[0, 1] - p[1, 0] + p[1, 1])
    return np.array(zi), np.array(zz)
