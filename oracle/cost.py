"""Expected entanglement of an unravelling as a function of the Kraus mixing (oracle).

For a noise channel {K_i} on the target qubit of a pure state with target reduced state
rho_q, a mixing U (K'_j = sum_i U_ji K_i) yields branches with weights
p_j = Tr(K'_j rho_q K'_j^dag) and target reduced states sigma_j = K'_j rho_q K'_j^dag / p_j
(the noisy-qubit : rest cut that the paper's unravelling minimises, Sec. "Problem statement
and main result").  The costs are

  f_lin(U) = sum_j p_j (1 - Tr sigma_j^2)            (linear entropy)
  f_R2(U)  = sum_j p_j (-log2 Tr sigma_j^2)          (Renyi-2 entropy)

with U = exp(i sum_k t_k L_k) U_ref over 16 Hermitian generators of u(4):
L_0..3 = E_kk, then for the pairs (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) the symmetric
E_jk + E_kj (L_4..9) and the antisymmetric i(E_kj - E_jk) (L_10..15).

The two-site reduction rho_q[s, s'] = sum_{a,t,b} theta[a,s,t,b] conj(theta[a,s',t,b]) is
taken in float64 from the (possibly complex64) tensor.

The reference gradient is reverse-mode differentiation of the same expression with torch
on the CPU in complex128 (a library primitive); tests also pin it with central finite
differences and with the optimum: at the Wootters mixing the linear cost equals C^2/2 and
its gradient vanishes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

KIND_LINEAR = 0
KIND_RENYI2 = 1
P_TINY = 1e-300


def generators() -> np.ndarray:
    g = np.zeros((16, 4, 4), dtype=np.complex128)
    for k in range(4):
        g[k, k, k] = 1.0
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for i, (j, k) in enumerate(pairs):
        g[4 + i, j, k] = g[4 + i, k, j] = 1.0
        g[10 + i, k, j] = 1j
        g[10 + i, j, k] = -1j
    return g


def unitary(params: np.ndarray, u_ref: np.ndarray) -> np.ndarray:
    h = np.einsum("k,kab->ab", params, generators())
    return scipy.linalg.expm(1j * h) @ u_ref


def pad_kraus(kraus: np.ndarray) -> np.ndarray:
    out = np.zeros((4, 2, 2), dtype=np.complex128)
    out[: kraus.shape[0]] = kraus
    return out


def rho_from_theta(theta: np.ndarray) -> np.ndarray:
    """theta[a][s][t][b] -> rho_q[s][s'] (float64 accumulation)."""
    t = theta.astype(np.complex128)
    return np.einsum("astb,aStb->sS", t, t.conj())


def cost(rho_q: np.ndarray, kraus: np.ndarray, u: np.ndarray, kind: int) -> float:
    kp = np.einsum("ji,iab->jab", u, pad_kraus(kraus))
    f = 0.0
    for k in kp:
        sig = k @ rho_q @ k.conj().T
        p = float(np.trace(sig).real)
        if p <= P_TINY:
            continue
        pur = float(np.trace(sig @ sig).real)
        if kind == KIND_LINEAR:
            f += p - pur / p
        else:
            f += -p * np.log2(pur / (p * p))
    return f


def cost_params(rho_q, kraus, params, u_ref, kind) -> float:
    return cost(rho_q, kraus, unitary(params, u_ref), kind)


def grad_torch(rho_q: np.ndarray, kraus: np.ndarray, params: np.ndarray, u_ref: np.ndarray,
               kind: int):
    """(f, df/dparams) by torch CPU autograd in complex128."""
    import torch
    th = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    gen = torch.tensor(generators())
    h = torch.einsum("k,kab->ab", th.to(torch.complex128), gen)
    u = torch.linalg.matrix_exp(1j * h) @ torch.tensor(u_ref)
    kp = torch.einsum("ji,iab->jab", u, torch.tensor(pad_kraus(kraus)))
    rho = torch.tensor(rho_q)
    f = torch.zeros((), dtype=torch.float64)
    for j in range(4):
        sig = kp[j] @ rho @ kp[j].conj().T
        p = torch.real(torch.trace(sig))
        if float(p.detach()) <= P_TINY:
            continue
        pur = torch.real(torch.trace(sig @ sig))
        if kind == KIND_LINEAR:
            f = f + p - pur / p
        else:
            f = f - p * torch.log2(pur / (p * p))
    f.backward()
    return float(f.detach()), th.grad.numpy().copy()


def grad_fd(rho_q, kraus, params, u_ref, kind, h=1e-4):
    g = np.zeros(16)
    for k in range(16):
        e = np.zeros(16)
        e[k] = h
        g[k] = (cost_params(rho_q, kraus, params + e, u_ref, kind)
                - cost_params(rho_q, kraus, params - e, u_ref, kind)) / (2 * h)
    return g


# --------------------------------------------------------------------- internal-bond cost
#
# The other reading of "the expected two-site entanglement": the entanglement across the
# two-site block's internal bond (a, s) : (t, b) after the noise event on site s.  Branch j
# of theta is theta_j = (K'_j on s) theta with weight p_j = ||theta_j||^2; its bond entropy is
# taken from the Gram matrix Gamma_j = theta_j theta_j^dag over (a, s):
#
#   f_lin^B(U) = sum_j p_j (1 - Tr Gamma_j^2 / p_j^2),   f_R2^B(U) = sum_j p_j (-log2 Tr Gamma_j^2 / p_j^2)
#
# computed here from the definition (branch tensors and their Gram matrices).


def bond_cost(theta: np.ndarray, kraus: np.ndarray, u: np.ndarray, kind: int) -> float:
    t = theta.astype(np.complex128)
    t = t / np.linalg.norm(t)
    kp = np.einsum("ji,iab->jab", u, pad_kraus(kraus))
    cl, cr = t.shape[0], t.shape[3]
    f = 0.0
    for k in kp:
        tj = np.einsum("xs,astb->axtb", k, t).reshape(2 * cl, 2 * cr)
        g = tj @ tj.conj().T
        p = float(np.trace(g).real)
        if p <= P_TINY:
            continue
        pur = float(np.trace(g @ g).real)
        if kind == KIND_LINEAR:
            f += p - pur / p
        else:
            f += -p * np.log2(pur / (p * p))
    return f


def bond_cost_params(theta, kraus, params, u_ref, kind) -> float:
    return bond_cost(theta, kraus, unitary(params, u_ref), kind)


def bond_grad_torch(theta: np.ndarray, kraus: np.ndarray, params: np.ndarray, u_ref: np.ndarray, kind: int):
    """(f^B, df^B/dparams) by torch CPU autograd in complex128 on the definition."""
    import torch
    th = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    gen = torch.tensor(generators())
    h = torch.einsum("k,kab->ab", th.to(torch.complex128), gen)
    u = torch.linalg.matrix_exp(1j * h) @ torch.tensor(u_ref)
    kp = torch.einsum("ji,iab->jab", u, torch.tensor(pad_kraus(kraus)))
    t = torch.tensor(theta.astype(np.complex128))
    t = t / torch.linalg.vector_norm(t)
    cl, cr = t.shape[0], t.shape[3]
    f = torch.zeros((), dtype=torch.float64)
    for j in range(4):
        tj = torch.einsum("xs,astb->axtb", kp[j], t).reshape(2 * cl, 2 * cr)
        g = tj @ tj.conj().T
        p = torch.real(torch.trace(g))
        if float(p.detach()) <= P_TINY:
            continue
        pur = torch.real(torch.trace(g @ g))
        if kind == KIND_LINEAR:
            f = f + p - pur / p
        else:
            f = f - p * torch.log2(pur / (p * p))
    f.backward()
    return float(f.detach()), th.grad.numpy().copy()


def bond_grad_fd(theta, kraus, params, u_ref, kind, h=1e-4):
    g = np.zeros(16)
    for k in range(16):
        e = np.zeros(16)
        e[k] = h
        g[k] = (bond_cost_params(theta, kraus, params + e, u_ref, kind)
                - bond_cost_params(theta, kraus, params - e, u_ref, kind)) / (2 * h)
    return g
