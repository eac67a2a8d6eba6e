"""Locally entanglement-optimal unravelling of a single-qubit channel (oracle).

Follows the paper step by step:

1. Reduction to the effective two-qubit problem (Sec. "Reduction to the effective two-qubit
   problem", Thm. 2): only the target qubit's reduced state rho_q matters; the effective
   state is Psi_eff = sqrt(rho_q) (target index x effective-partner index), a purification
   of rho_q whose partner basis differs from the paper's U S only by a unitary on the
   partner, which leaves the optimum unchanged.
2. Induced decomposition phi = [vec(K_i Psi_eff)]_i (matrix notation of ensembles, appendix
   "Ensemble decomposition matrix formulation"); SVD(phi) = U_phi Sigma V_phi^dag gives the
   sub-normalised eigen-decomposition v = U_phi Sigma and U_0 = V_phi^dag (Sec. "Optimal
   unraveling unitary").
3. Wootters' Step 1 (appendix, practical version): tau = v^dag v~ with v~ = (Y x Y) v*, a
   complex symmetric matrix; its Takagi factorisation tau = U_T Sigma_tau U_T^T gives
   x = v U_T with x^dag x~ = diag(lambda_R) (eigenvalues of R, sorted descending).
4. Step 2: y = x U_2^dag with U_2 = diag(1, i, i, i).
5. Step 3: M = y^dag y~ - C y^dag y, Q_R from the eigen-decomposition of Re(M),
   U_3 = H_4 Q_R^T, z = y U_3^dag.
6. Separable case (C = 0): z = x diag(e^{i theta_j}) H_4 with the trapezoid angles.
7. Back to Kraus operators: z = phi W with W = V_phi[:, :rank] U_T E (E the 4x4 map of
   steps 4-6 restricted to the first ``rank`` rows); K'_j = sum_i W_ij K_i.

Readings taken where the text is garbled or silent (each also listed in the design notes):
* mixing convention K'_j = sum_i U_ji K_i, i.e. U = W^T (worked dephasing example);
* v from the SVD of phi (not from eigh(rho_eff) and square roots of clipped eigenvalues);
* work in the numerical rank of phi (sigma_j > 1e-12 sigma_1) and zero-pad x to 4 columns
  (footnote on rank < 4);
* Takagi through the real symmetric embedding [[A, B], [B, -A]] of tau = A + iB (positive
  eigenvalues sigma with eigenvectors [a; b] give Takagi vectors a + ib); null directions of
  tau are conj(null(tau)) with the phase fixed so that the largest-modulus entry of the
  corresponding column of v U_T is real positive;
* lambda_R sorted descending, ties by index; Q_R columns in ascending eigenvalue order, each
  signed so its largest-modulus entry (lowest index on ties) is positive;
* separable angles: theta_1 = 0, theta_4 = pi/2, 2 theta_2 = pi - arcsin(h / lambda_2),
  2 theta_3 = arg(lambda_4 - lambda_1 - lambda_2 e^{2i theta_2}) (closing side of the
  polygon sum_j lambda_j e^{2i theta_j} = 0), all-equal lambdas -> (0, pi/4, pi/2, 3pi/4);
  z carries the factor 1/2 so that it is a unitary image of x.

Parity pins: Choi-state closed forms for dephasing, amplitude damping and depolarizing
noise; the amplitude-damping computational-Schmidt-basis concurrence; E_av == EoF on random
inputs; completeness of the returned Kraus set; brute-force search never below EoF.
"""
from __future__ import annotations

import numpy as np

MODE_ORTHOGONAL = 0
MODE_FIXED = 1
MODE_HAAR_OPT = 2
MODE_OPTIMAL = 3
MODE_LEAST_UNITARY = 4

YY = np.kron(np.array([[0, -1j], [1j, 0]]), np.array([[0, -1j], [1j, 0]])).real.astype(np.complex128)
H4 = 0.5 * np.array([[1, 1, 1, 1], [1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]],
                    dtype=np.complex128)
RANK_TOL = 1e-12


def binary_entropy(x: float) -> float:
    """h(x) = -x log2 x - (1-x) log2 (1-x), h(0) = h(1) = 0."""
    out = 0.0
    for t in (x, 1.0 - x):
        if t > 0.0:
            out -= t * np.log2(t)
    return out


def eof_from_concurrence(c: float) -> float:
    """Hill-Wootters: E_oF = h((1 + sqrt(1 - C^2)) / 2)."""
    c = min(max(c, 0.0), 1.0)
    return binary_entropy(0.5 * (1.0 + np.sqrt(max(0.0, 1.0 - c * c))))


def spin_flip(v: np.ndarray) -> np.ndarray:
    """Column-wise spin flip (Y x Y) v* of two-qubit vectors."""
    return YY @ v.conj()


def pure_entropy(psi: np.ndarray) -> float:
    """Entanglement entropy (base 2) of a normalised two-qubit vector, target:partner."""
    s = np.linalg.svd(psi.reshape(2, 2), compute_uv=False)
    return binary_entropy(float(s[0] ** 2))


def effective_state(rho_q: np.ndarray) -> np.ndarray:
    """Psi_eff = the positive square root of rho_q; rows = target, columns = partner."""
    w, u = np.linalg.eigh(rho_q)
    w = np.clip(w, 0.0, None)
    return (u * np.sqrt(w)[None, :]) @ u.conj().T


def induced_decomposition(rho_q: np.ndarray, kraus: np.ndarray) -> np.ndarray:
    """phi = [vec(K_i Psi_eff)]_i, 4 x r, vec row-major (target index major)."""
    psi = effective_state(rho_q)
    return np.stack([(k @ psi).reshape(4) for k in kraus], axis=1)


def takagi(tau: np.ndarray):
    """Takagi factorisation of a complex symmetric matrix: returns (sigma, U) with
    tau = U diag(sigma) U^T, sigma descending, U unitary.

    Positive sigma come from the real symmetric embedding [[A, B], [B, -A]] (tau = A + iB):
    an eigenvector [a; b] with eigenvalue sigma > 0 gives tau conj(a + ib) = sigma (a + ib).
    Null directions are conj(null(tau)); they are orthogonal to the range block because
    tau is symmetric.  Column signs / phases are left to the caller to pin."""
    m = tau.shape[0]
    a, b = tau.real, tau.imag
    w, q = np.linalg.eigh(np.block([[a, b], [b, -a]]))
    smax = max(float(np.max(np.abs(w))), 1e-300)
    cols, sig = [], []
    for idx in np.argsort(-w, kind="stable")[:m]:
        if w[idx] <= RANK_TOL * smax:
            break
        u = q[:m, idx] + 1j * q[m:, idx]
        cols.append(u / np.linalg.norm(u))
        sig.append(float(w[idx]))
    k = len(cols)
    if k < m:
        _, _, vh = np.linalg.svd(tau)
        for j in range(k, m):
            cols.append(vh[j].copy())       # rows of V^dag with sigma = 0 are conj(null)
            sig.append(0.0)
    return np.array(sig), np.stack(cols, axis=1)


def first_argmax(a: np.ndarray) -> int:
    """Index of the largest-modulus entry; near-ties (relative 1e-12) go to the lowest
    index."""
    m = np.abs(a)
    mx = float(np.max(m))
    return int(np.nonzero(m >= mx * (1.0 - 1e-12))[0][0])


def pin_takagi_columns(v: np.ndarray, ut: np.ndarray, sig: np.ndarray) -> np.ndarray:
    """Fix the residual freedom of Takagi vectors through their image x_j = v u_j:
    sigma_j > 0 (sign freedom): the largest-modulus entry of x_j gets a non-negative real
    part; sigma_j = 0 (phase freedom): that entry is made real positive."""
    ut = ut.copy()
    x = v @ ut
    for j in range(ut.shape[1]):
        i = first_argmax(x[:, j])
        e = x[i, j]
        if abs(e) == 0.0:
            continue
        if sig[j] > 0.0:
            if e.real < 0.0 or (e.real == 0.0 and e.imag < 0.0):
                ut[:, j] = -ut[:, j]
        else:
            ut[:, j] = ut[:, j] * (abs(e) / e)
    return ut


def sign_fix_columns(q: np.ndarray) -> np.ndarray:
    """Each real column signed so its largest-|.| entry (lowest index on ties) is
    positive."""
    q = q.copy()
    for j in range(q.shape[1]):
        i = first_argmax(q[:, j])
        if q[i, j] < 0:
            q[:, j] = -q[:, j]
    return q


def separable_angles(lam: np.ndarray) -> np.ndarray:
    """theta_1..4 with sum_j lambda_j e^{2 i theta_j} = 0 (lambda descending, separable)."""
    l1, l2, l3, l4 = (float(x) for x in lam)
    if l1 - l4 <= 1e-15 * max(l1, 1e-300):
        return np.array([0.0, np.pi / 4, np.pi / 2, 3 * np.pi / 4])
    base = l1 - l4
    s = 0.5 * (base + l2 + l3)
    area2 = max(0.0, s * (s - base) * (s - l2) * (s - l3))
    h = 2.0 / base * np.sqrt(area2)
    two_t2 = np.pi - np.arcsin(min(1.0, h / l2)) if l2 > 0 else np.pi
    closing = (l4 - l1) - l2 * np.exp(1j * two_t2)
    two_t3 = float(np.angle(closing)) if abs(closing) > 0 else 0.0
    return np.array([0.0, 0.5 * two_t2, 0.5 * two_t3, np.pi / 2])


def optimal_mixing(rho_q: np.ndarray, kraus: np.ndarray):
    """The locally entanglement-optimal mixing for noise ``kraus`` on a qubit with reduced
    state ``rho_q`` (normalised).

    Returns dict with W (r x 4, K'_j = sum_i W_ij K_i, rows orthonormal so the K'_j form a
    complete Kraus set), p (4 branch weights), C (concurrence of rho_eff), eof, lam_R (4),
    separable flag, z (4 x 4 sub-normalised branch vectors of the effective two-qubit state)
    and the intermediate objects of the steps.
    """
    r = kraus.shape[0]
    phi = induced_decomposition(rho_q, kraus)                      # step 2
    uphi, sphi, vphih = np.linalg.svd(phi, full_matrices=True)     # phi = U S V^dag
    vphi = vphih.conj().T                                          # r x r
    rank = int(np.sum(sphi > RANK_TOL * sphi[0])) if sphi[0] > 0 else 0
    if rank == 0:
        raise ValueError("zero state")
    v = uphi[:, :rank] * sphi[None, :rank]                         # 4 x rank
    tau = v.conj().T @ spin_flip(v)                                # step 3
    tau = 0.5 * (tau + tau.T)
    sig, ut = takagi(tau)
    ut = pin_takagi_columns(v, ut, sig)
    x = np.zeros((4, 4), dtype=np.complex128)
    x[:, :rank] = v @ ut
    lam = np.zeros(4)
    lam[:rank] = sig
    conc = max(0.0, lam[0] - lam[1] - lam[2] - lam[3])
    separable = not (lam[0] - lam[1] - lam[2] - lam[3] > 0.0)
    if not separable:
        u2dag = np.diag([1, -1j, -1j, -1j])                          # step 4
        y = x @ u2dag
        m = y.conj().T @ spin_flip(y) - conc * (y.conj().T @ y)      # step 5
        mr = 0.5 * (m.real + m.real.T)
        _, qr = np.linalg.eigh(mr)
        qr = sign_fix_columns(qr)
        e = u2dag @ qr @ H4.T
    else:
        th = separable_angles(lam)                                   # step 6
        e = np.diag(np.exp(1j * th)) @ H4
    # step 7: z = phi W.  Rows rank..r-1 of E complete W to orthonormal rows on the null
    # space of phi (linearly dependent Kraus operators / rank-deficient rho_q); they do not
    # change z.
    w = vphi[:, :rank] @ ut @ e[:rank, :]
    if rank < r:
        w = w + vphi[:, rank:r] @ e[rank:r, :]
    z = phi @ w
    p = np.sum(np.abs(z) ** 2, axis=0)
    return dict(W=w, p=p, C=conc, eof=eof_from_concurrence(conc), lam_R=lam,
                separable=separable, z=z, phi=phi, v=v, tau=tau, x=x, rank=rank)


def haar_optimal_u(r: int) -> np.ndarray:
    """The mixing of the Haar Optimal unravelings (table of unravelings, Sec. "Noisy random
    circuits"; appendix "Some common unravelings"): the Orthogonal Kraus set rotated by the
    Hadamard matrix H (two operators: dephasing, amplitude damping) or, for four operators
    (depolarizing), by the 4 x 4 matrix the appendix prints (H (x) H with its two middle rows
    exchanged: the same operators in the printed branch order); one operator is left alone.
    Returned as 4 x r, zero rows past r."""
    h = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
    h4 = 0.5 * np.array([[1, 1, 1, 1], [1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]], dtype=np.complex128)
    mats = {1: np.ones((1, 1), dtype=np.complex128), 2: h, 4: h4}
    if r not in mats:
        raise ValueError(f"the Haar Optimal mixing is defined for 1, 2 or 4 Kraus operators, not {r}")
    u = np.zeros((4, r), dtype=np.complex128)
    u[:r] = mats[r]
    return u


def least_unitary_w(kraus: np.ndarray) -> np.ndarray:
    """The least unitary unraveling (appendix "Vectorized Kraus operators and the least
    unitary unraveling"): the locally entanglement-optimal mixing for the maximally mixed
    reduced state I/2, i.e. Wootters' optimal decomposition of the channel's normalised Choi
    state; it does not depend on the state it is applied to."""
    return optimal_mixing(np.eye(2, dtype=np.complex128) / 2.0, kraus)["W"]


def mixing(rho_q: np.ndarray, kraus: np.ndarray, mode: int, fixed_u=None) -> np.ndarray:
    """W (r x 4) for the requested unravelling mode.

    ORTHOGONAL:    the channel's own Kraus operators (padded with zero operators to 4);
    FIXED:         K'_j = sum_i U_ji K_i for a caller-given 4 x r matrix U;
    HAAR_OPT:      FIXED with the Haar Optimal mixing of the channel's rank;
    OPTIMAL:       the locally entanglement-optimal mixing above;
    LEAST_UNITARY: the optimal mixing of the channel's Choi state (state independent).
    """
    r = kraus.shape[0]
    if mode == MODE_ORTHOGONAL:
        w = np.zeros((r, 4), dtype=np.complex128)
        w[:, :r] = np.eye(r)
        return w
    if mode == MODE_FIXED:
        return np.asarray(fixed_u, dtype=np.complex128).T.copy()
    if mode == MODE_HAAR_OPT:
        return haar_optimal_u(r).T.copy()
    if mode == MODE_OPTIMAL:
        return optimal_mixing(rho_q, kraus)["W"]
    if mode == MODE_LEAST_UNITARY:
        return least_unitary_w(kraus)
    raise ValueError(f"unknown mode {mode}")


def mixed_kraus(kraus: np.ndarray, w: np.ndarray) -> np.ndarray:
    """K'_j = sum_i W_ij K_i  (4 x 2 x 2)."""
    return np.einsum("ij,iab->jab", w, kraus)


def average_entanglement(rho_q: np.ndarray, kraus_prime: np.ndarray):
    """(p_j, E_av) of the ensemble induced by K'_j on the effective two-qubit state."""
    psi = effective_state(rho_q)
    ps, e = [], 0.0
    for k in kraus_prime:
        z = (k @ psi).reshape(4)
        pj = float(np.vdot(z, z).real)
        ps.append(pj)
        if pj > 1e-300:
            e += pj * pure_entropy(z / np.sqrt(pj))
    return np.array(ps), e


def concurrence_hill_wootters(rho: np.ndarray) -> float:
    """C(rho) from R = sqrt(sqrt(rho) rho~ sqrt(rho)) (appendix on Wootters' decomposition),
    computed with Hermitian square roots."""
    def psd_sqrt(a):
        w, u = np.linalg.eigh(0.5 * (a + a.conj().T))
        return (u * np.sqrt(np.clip(w, 0, None))[None, :]) @ u.conj().T
    sr = psd_sqrt(rho)
    rt = YY @ rho.conj() @ YY
    lam = np.sort(np.sqrt(np.clip(np.linalg.eigvalsh(sr @ rt @ sr), 0, None)))[::-1]
    return max(0.0, lam[0] - lam[1] - lam[2] - lam[3])
