"""MPS trajectories with bond-dimension truncation (oracle).

A plain textbook implementation of the MPS-based trajectory sampling of the paper (Sec.
"Details of MPS-based trajectory sampling"): site tensors A^[k]_s (eq. def_MPS) stored as
(2, d_k, d_{k+1}) arrays, an orthogonality centre moved with QR factorisations, and the
local layering (Trunc o N^{x2} o U per gate, Sec. "Details of MPS-based trajectory
sampling"):

  1. contract the two site tensors of the pair and the gate into theta;
  2. for each noise event on the pair (lower qubit first), unravel with the qubit's
     reduced state, compute p_j, draw j, apply K'_j / sqrt(p_j) to theta (Alg. 1);
  3. SVD of theta across the pair's bond, keep the min(chi, #) largest singular values,
     record the discarded weight eps = sum_{i > chi} s_i^2 / sum_i s_i^2 (eq.
     MPS_truncation_error), renormalise, split into A^[q] (left-orthonormal) and the new
     centre A^[q+1].

Noise on a qubit left idle by a layer is applied to the centre tensor at that site.  The
sweep order is the one of ``sv.sweep_ops``.

Pinned by: equality with the statevector trajectory (same seeds) when chi >= 2^(n/2), norm
1 after every step, and the Eckart-Young identity ||psi - P psi||^2 = eps for one bond.
"""
from __future__ import annotations

import numpy as np

from . import rng as _rng
from . import sv as _sv
from . import unravel as _unr


class MPS:
    def __init__(self, n: int):
        self.n = n
        self.t = []
        for _ in range(n):
            a = np.zeros((2, 1, 1), dtype=np.complex128)
            a[0, 0, 0] = 1.0
            self.t.append(a)
        self.centre = 0

    # ----------------------------------------------------------------- canonical form
    def _hop_right(self, j: int):
        a = self.t[j]
        s, dl, dr = a.shape
        q, r = np.linalg.qr(a.reshape(s * dl, dr))
        self.t[j] = q.reshape(s, dl, q.shape[1])
        self.t[j + 1] = np.einsum("kb,sbc->skc", r, self.t[j + 1])
        self.centre = j + 1

    def _hop_left(self, j: int):
        a = self.t[j]
        s, dl, dr = a.shape
        m = a.transpose(1, 0, 2).reshape(dl, s * dr)
        q, r = np.linalg.qr(m.conj().T)            # m = r^dag q^dag
        k = q.shape[1]
        self.t[j] = q.conj().T.reshape(k, s, dr).transpose(1, 0, 2)
        self.t[j - 1] = np.einsum("sab,bk->sak", self.t[j - 1], r.conj().T)
        self.centre = j - 1

    def move_centre(self, target: int):
        while self.centre < target:
            self._hop_right(self.centre)
        while self.centre > target:
            self._hop_left(self.centre)

    # ----------------------------------------------------------------- dense conversion
    def to_vector(self) -> np.ndarray:
        v = self.t[0][:, 0, :]                                   # (2, d1)
        for k in range(1, self.n):
            v = np.einsum("xb,sbc->xsc", v, self.t[k]).reshape(-1, self.t[k].shape[2])
        return v[:, 0]

    def bond_dims(self):
        return [a.shape[2] for a in self.t[:-1]]


def _event_on_theta(theta, which, kraus, mode, u, fixed_u, record, q, replay=None):
    """Noise event on the first (which=0) or second (which=1) physical index of theta."""
    axes = (1, 2, 3) if which == 0 else (0, 2, 3)
    rho = np.tensordot(theta, theta.conj(), axes=(axes, axes))
    rho = rho / np.trace(rho).real
    w = _sv.choose_mixing(rho, kraus, mode, fixed_u, replay)
    kp = _unr.mixed_kraus(kraus, w)
    sub = "xs,stac->xtac" if which == 0 else "yt,stac->syac"
    outs = [np.einsum(sub, k, theta) for k in kp]
    norm = np.vdot(theta, theta).real
    p = np.array([np.vdot(o, o).real / norm for o in outs])
    j = _rng.sample_branch(p, u)
    if record is not None:
        record.append(dict(q=q, p=p, j=j, W=w))
    return outs[j] / np.sqrt(p[j] * norm)


def gate_step(m: MPS, l: int, q: int, circuit, chi: int, traj: int, seed: int, mode,
              fixed_u=None, record=None, replay=None, spectra=None):
    """One trajectory gate-step on the pair (q, q+1); returns the discarded weight.  If
    `spectra` is a list, the full singular-value spectrum of the split (before truncation)
    is appended to it."""
    m.move_centre(q)
    theta = np.einsum("sab,tbc->stac", m.t[q], m.t[q + 1])
    g = circuit.gate(l, q).reshape(2, 2, 2, 2)
    theta = np.einsum("xyst,stac->xyac", g, theta)
    for which, x in ((0, q), (1, q + 1)):
        ch = int(circuit.events[l, x])
        if ch >= 0:
            u = _rng.uniform(seed, traj, l, x)
            theta = _event_on_theta(theta, which, circuit.kraus(ch), mode, u, fixed_u,
                                    record, x, replay)
    _, _, dl, dr = theta.shape
    mat = theta.transpose(0, 2, 1, 3).reshape(2 * dl, 2 * dr)
    u_, s, vh = np.linalg.svd(mat, full_matrices=False)
    if spectra is not None:
        spectra.append(s.copy())
    tot = float(np.sum(s ** 2))
    d = min(chi, s.size)
    kept = float(np.sum(s[:d] ** 2))
    eps = (tot - kept) / tot
    s = s[:d] / np.sqrt(kept)
    m.t[q] = u_[:, :d].reshape(2, dl, d)
    m.t[q + 1] = (s[:, None] * vh[:d]).reshape(d, 2, dr).transpose(1, 0, 2)
    m.centre = q + 1
    return eps


def idle_event(m: MPS, l: int, q: int, circuit, traj: int, seed: int, mode, fixed_u=None,
               record=None, replay=None):
    m.move_centre(q)
    a = m.t[q]
    rho = np.tensordot(a, a.conj(), axes=((1, 2), (1, 2)))
    rho = rho / np.trace(rho).real
    kraus = circuit.kraus(int(circuit.events[l, q]))
    w = _sv.choose_mixing(rho, kraus, mode, fixed_u, replay)
    kp = _unr.mixed_kraus(kraus, w)
    outs = [np.einsum("xs,sab->xab", k, a) for k in kp]
    norm = np.vdot(a, a).real
    p = np.array([np.vdot(o, o).real / norm for o in outs])
    j = _rng.sample_branch(p, _rng.uniform(seed, traj, l, q))
    if record is not None:
        record.append(dict(q=q, p=p, j=j, W=w))
    m.t[q] = outs[j] / np.sqrt(p[j] * norm)


def trajectory(circuit, chi: int, traj: int, seed: int, mode=_unr.MODE_OPTIMAL,
               fixed_u=None, layers=None, record=None, layer_range=None, m: MPS = None,
               replay=None, spectra=None):
    """Run one trajectory; returns (MPS, list of per-gate discarded weights)."""
    if m is None:
        m = MPS(circuit.n)
    eps = []
    rng_l = range(circuit.depth if layers is None else layers) if layer_range is None else layer_range
    for l in rng_l:
        for kind, q in _sv.sweep_ops(circuit, l):
            if kind == "gate":
                eps.append(gate_step(m, l, q, circuit, chi, traj, seed, mode, fixed_u, record,
                                     replay, spectra))
            else:
                idle_event(m, l, q, circuit, traj, seed, mode, fixed_u, record, replay)
    return m, eps


def truncate_sweep(m: MPS, chi: int):
    """Truncation of every bond to chi by a left-to-right sweep (the approximation
    subprocedure applied to all bonds): with the centre at site k, the SVD of the centre
    reshaped (2 d_k) x d_(k+1) keeps its top-chi singular values, renormalised, and moves the
    centre to k + 1.  Returns the list of discarded weights (one per bond)."""
    m.move_centre(0)
    eps = []
    for k in range(m.n - 1):
        a = m.t[k]
        s_, dl, dr = a.shape
        u_, s, vh = np.linalg.svd(a.reshape(s_ * dl, dr), full_matrices=False)
        tot = float(np.sum(s ** 2))
        d = min(chi, s.size)
        kept = float(np.sum(s[:d] ** 2))
        eps.append((tot - kept) / tot if tot > 0 else 0.0)
        s = s[:d] / np.sqrt(kept)
        m.t[k] = u_[:, :d].reshape(s_, dl, d)
        m.t[k + 1] = np.einsum("kb,sbc->skc", s[:, None] * vh[:d], m.t[k + 1])
        m.centre = k + 1
    m.move_centre(0)
    return eps


def trajectory_global(circuit, chi: int, traj: int, seed: int, mode=_unr.MODE_OPTIMAL,
                      fixed_u=None, layers=None, record=None, replay=None):
    """Global layering (Sec. "Details of MPS-based trajectory sampling"): every layer applies
    its gates and its noise with no truncation (the bond dimension of the acted bonds may
    reach twice its value), then truncates all bonds to chi with one sweep.  Returns (MPS,
    discarded weights per layer)."""
    m = MPS(circuit.n)
    eps = []
    for l in range(circuit.depth if layers is None else layers):
        trajectory(circuit, 1 << 30, traj, seed, mode, fixed_u, record=record, layer_range=[l], m=m,
                   replay=replay)
        eps.append(truncate_sweep(m, chi))
    return m, eps


def born_sample(m: MPS, n_samples: int, seed: int, traj: int):
    """Bitstrings drawn from the Born distribution |<x|psi>|^2 of the MPS (Lemma on output
    distribution sampling: sampling each trajectory samples the mixture), site by site from
    the conditional probabilities: with the centre at site 0 the rest is right-orthonormal, so
    after outcomes s_0..s_(k-1) with the left vector v, p(s_k = s) is proportional to
    ||v A_k^s||^2.  The uniform of site k of sample i is the counter draw keyed by (traj,
    i, k) of `seed`; s_k = 0 when u < p_0 / (p_0 + p_1).  Returns (bits [n_samples][n],
    probability of each drawn bitstring)."""
    m.move_centre(0)
    bits = np.zeros((n_samples, m.n), dtype=np.uint8)
    probs = np.ones(n_samples)
    for i in range(n_samples):
        v = np.ones(1, dtype=np.complex128)
        for k in range(m.n):
            w = [v @ m.t[k][s] for s in (0, 1)]
            p = [float(np.vdot(x, x).real) for x in w]
            u = _rng.uniform(seed, traj, i, k)
            s = 0 if u < p[0] / (p[0] + p[1]) else 1
            bits[i, k] = s
            probs[i] *= p[s] / (p[0] + p[1])
            v = w[s] / np.sqrt(p[s])
    return bits, probs


def z_expectations(m: MPS):
    """<Z_i>, <Z_i Z_{i+1}> by sweeping the centre left to right."""
    n = m.n
    zs = np.array([1.0, -1.0])
    zi, zz = [], []
    m.move_centre(0)
    for i in range(n):
        m.move_centre(i)
        a = m.t[i]
        w = np.sum(np.abs(a) ** 2, axis=(1, 2))
        zi.append(float(np.dot(zs, w) / w.sum()))
        if i + 1 < n:
            th = np.einsum("sab,tbc->stac", a, m.t[i + 1])
            w2 = np.sum(np.abs(th) ** 2, axis=(2, 3))
            zz.append(float(np.einsum("s,t,st->", zs, zs, w2) / w2.sum()))
    return np.array(zi), np.array(zz)
