"""Trotterised time-independent Lindbladian evolution (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. "Time-independent Lindbladian systems" and the appendix "Exact decomposition of
Trotterized Lindbladian evolutions", in the paper's steps:

* vectorisation |rho>> = (rho (x) I)|Omega>, so that (A (x) B)|rho>> = |A rho B^T>> and the
  Lindbladian is L = -i (H (x) I - I (x) H^T) + sum_j gamma_j (c_j (x) c_j^* - 1/2 c_j^dag c_j
  (x) I - 1/2 I (x) c_j^T c_j^*);
* Trotter step of length dt: a layer of exp(-i H_(i,i+1) dt) on the pairs of one parity, the
  jump processes of every site for dt/2, a layer on the pairs of the other parity, the jump
  processes for dt/2 again (the factors in the time order of the text);
* the jump channel e^{L_jump tau} reshaped into its Choi matrix, whose eigendecomposition
  gives an orthogonal Kraus set: K_i = sqrt(lambda_i) reshape(v_i);
* the exact evolution exp(L t) of the whole chain (a few qubits) for the Trotter error.

Pinned by: the two remarks of the appendix on typical jump operators (c = |0><0| gives
dephasing with p = 1 - exp(-gamma dt / 2) in its I / Z form; c = |0><1| gives amplitude
damping with gamma_AD = 1 - exp(-gamma dt) in its usual form), trace preservation, and the
first-order convergence of the Trotterised density matrix to exp(L t).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from . import dm as _dm

_I2 = np.eye(2, dtype=np.complex128)


def jump_superoperator(c: np.ndarray, gamma: float) -> np.ndarray:
    """gamma (c (x) c^* - 1/2 c^dag c (x) I - 1/2 I (x) c^T c^*), 4 x 4."""
    c = np.asarray(c, dtype=np.complex128)
    return gamma * (np.kron(c, c.conj()) - 0.5 * np.kron(c.conj().T @ c, _I2) - 0.5 * np.kron(_I2, c.T @ c.conj()))


def choi_of_superoperator(s: np.ndarray) -> np.ndarray:
    """Reshuffle of a one-qubit superoperator S[(a,b),(c,d)] (acting as rho_cd -> rho_ab) into
    its Choi matrix J[(a,c),(b,d)] = sum_k K_ac K_bd^* (for S = sum_k K (x) K^*)."""
    return np.asarray(s).reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)


def jump_kraus(jumps, tau: float, rel_tol: float = 1e-14) -> np.ndarray:
    """Kraus operators of exp(sum_j L_j tau) for single-site jumps [(c_j, gamma_j)]: the
    eigenvectors of the Choi matrix with their eigenvalues, descending, zero eigenvalues (below
    rel_tol of the largest) left out.  Convention (an eigenvector's phase is free): each
    operator's largest-modulus entry, the first one in row-major order among entries within a
    factor 1 + 1e-12 of it, is made real positive."""
    s = sum(jump_superoperator(c, g) for c, g in jumps)
    j = choi_of_superoperator(expm(s * tau))
    j = 0.5 * (j + j.conj().T)
    w, v = np.linalg.eigh(j)
    order = np.argsort(-w, kind="stable")
    w, v = w[order], v[:, order]
    keep = w > rel_tol * w[0]
    out = []
    for i in np.nonzero(keep)[0]:
        vi = v[:, i]
        a = np.abs(vi)
        big = int(np.nonzero(a * (1.0 + 1e-12) >= a.max())[0][0])
        out.append(np.sqrt(w[i]) * (vi * np.conj(vi[big]) / a[big]).reshape(2, 2))
    return np.stack(out)


def trotter_gate(h: np.ndarray, dt: float) -> np.ndarray:
    return expm(-1j * np.asarray(h, dtype=np.complex128) * dt)


def circuit(model):
    """The model's Trotterised noisy brickwork circuit, built with this module's gates and
    Kraus operators."""
    from paper_2508_05745_amd import inputs as I
    gates = {q: trotter_gate(model.pair_hamiltonian(q), model.dt) for q in range(model.n - 1)}
    return I.lindblad_circuit(model, gates, jump_kraus(model.jumps, model.dt / 2))


def _site_op(op: np.ndarray, q: int, n: int) -> np.ndarray:
    return np.kron(np.kron(np.eye(2 ** q), op), np.eye(2 ** (n - q - 1)))


def lindbladian(model) -> np.ndarray:
    """The vectorised Lindbladian of the whole chain (4^n x 4^n)."""
    n = model.n
    d = 2 ** n
    h = np.zeros((d, d), dtype=np.complex128)
    for q in range(n - 1):
        h += np.kron(np.kron(np.eye(2 ** q), model.pair_hamiltonian(q)), np.eye(2 ** (n - q - 2)))
    eye = np.eye(d, dtype=np.complex128)
    L = -1j * (np.kron(h, eye) - np.kron(eye, h.T))
    for q in range(n):
        for c, g in model.jumps:
            cq = _site_op(np.asarray(c, dtype=np.complex128), q, n)
            L += g * (np.kron(cq, cq.conj()) - 0.5 * np.kron(cq.conj().T @ cq, eye) - 0.5 * np.kron(eye, cq.T @ cq.conj()))
    return L


def exact_state(model, t: float) -> np.ndarray:
    """exp(L t) applied to |0..0><0..0| (2^n x 2^n)."""
    d = 2 ** model.n
    rho0 = np.zeros((d, d), dtype=np.complex128)
    rho0[0, 0] = 1.0
    return (expm(lindbladian(model) * t) @ rho0.reshape(-1)).reshape(d, d)


def trotter_state(model) -> np.ndarray:
    """Exact density matrix of the Trotterised circuit after all its steps."""
    return _dm.run(circuit(model))
