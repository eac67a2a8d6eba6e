"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module only *describes problems*: random two-qubit gates, single-qubit channels given
by their Kraus operators, brickwork circuit tables and random two-site states.  It holds
none of the simulation method's arithmetic (no unravelling, no contraction, no sampling).

Conventions (both the oracle and the HIP path read them from here):

* qubit ``q`` of an ``n``-qubit chain is MPS site ``q``; in a dense state vector qubit 0 is
  the most significant bit.
* a two-qubit gate on the pair ``(q, q+1)`` is a 4x4 matrix on the basis index ``2*s + t``
  with ``s`` the state of qubit ``q`` and ``t`` that of qubit ``q+1``.
* brickwork layer ``l`` (0-based) acts on the pairs ``(p, p+1), (p+2, p+3), ...`` with
  ``p = l % 2``; the first layer therefore starts at qubit 0.
* a channel is a stack ``[r][2][2]`` of Kraus operators (r <= 4).  Noise events are listed
  per ``(layer, qubit)`` as an index into the channel table, -1 meaning no noise.

Channel parametrisations follow the paper's section on common unravelings (depolarizing
with rate p, dephasing with rate p, amplitude damping with rate gamma).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

# ----------------------------------------------------------------------------- gates


def haar_unitary(rng: np.random.Generator, d: int = 4) -> np.ndarray:
    """Haar-random d x d unitary: QR of a complex Ginibre matrix with the phases of R's
    diagonal moved into Q (Mezzadri's recipe)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return (q * ph[None, :]).astype(np.complex128)


# ----------------------------------------------------------------------------- channels

_I = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def depolarizing(p: float) -> np.ndarray:
    """rho -> (1-p) rho + p I/2 as the four rescaled Paulis."""
    return np.stack([np.sqrt(1 - 3 * p / 4) * _I, np.sqrt(p) / 2 * _X,
                     np.sqrt(p) / 2 * _Y, np.sqrt(p) / 2 * _Z])


def dephasing(p: float) -> np.ndarray:
    """rho -> (1-p/2) rho + (p/2) Z rho Z (mixed-unitary form)."""
    return np.stack([np.sqrt(1 - p / 2) * _I, np.sqrt(p / 2) * _Z])


def amplitude_damping(gamma: float) -> np.ndarray:
    """The usual two-operator form diag(1, sqrt(1-gamma)), sqrt(gamma)|0><1|."""
    k0 = np.array([[1, 0], [0, np.sqrt(1 - gamma)]], dtype=np.complex128)
    k1 = np.array([[0, np.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    return np.stack([k0, k1])


def random_channel(r: int, seed: int) -> np.ndarray:
    """A seeded random single-qubit channel with r Kraus operators: the r 2 x 2 blocks of a
    random 2r x 2 isometry (QR of a complex Gaussian matrix), so that sum K^dag K = I."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((2 * r, 2)) + 1j * rng.standard_normal((2 * r, 2))
    q, _ = np.linalg.qr(z)
    return q.reshape(r, 2, 2).astype(np.complex128)


def compose(first: np.ndarray, second: np.ndarray) -> np.ndarray:
    """Kraus set of ``second o first``: all products K2_j K1_i (j major)."""
    return np.stack([k2 @ k1 for k2 in second for k1 in first])


# ----------------------------------------------------------------------------- circuits


def layer_pairs(n: int, layer: int) -> List[int]:
    """Left qubits of the pairs acted on by brickwork layer ``layer``."""
    p = layer % 2
    return list(range(p, n - 1, 2))


@dataclasses.dataclass
class Circuit:
    """A noisy brickwork circuit on an open chain.

    gates:    [depth][max_pairs][4][4] complex128; slot i of layer l is the pair
              (p + 2i, p + 2i + 1) with p = l % 2.
    channels: [n_channels][4][2][2] complex128, Kraus stacks zero-padded to 4.
    n_kraus:  [n_channels] number of meaningful Kraus operators per channel.
    events:   [depth][n] int32 channel id of the noise applied to qubit q in layer l
              (-1 = none).  Noise on a gate's qubits follows that gate; noise on an idle
              qubit is applied when the sweep passes it.
    """
    n: int
    depth: int
    gates: np.ndarray
    channels: np.ndarray
    n_kraus: np.ndarray
    events: np.ndarray
    name: str = ""

    def pairs(self, layer: int) -> List[int]:
        return layer_pairs(self.n, layer)

    def gate(self, layer: int, q: int) -> np.ndarray:
        return self.gates[layer, (q - layer % 2) // 2]

    def kraus(self, ch: int) -> np.ndarray:
        return self.channels[ch, : self.n_kraus[ch]]

    @property
    def n_gates(self) -> int:
        return sum(len(self.pairs(l)) for l in range(self.depth))


def _pad_channels(chs: List[np.ndarray]):
    tab = np.zeros((len(chs), 4, 2, 2), dtype=np.complex128)
    nk = np.zeros(len(chs), dtype=np.int32)
    for i, k in enumerate(chs):
        if k.shape[0] > 4:
            raise ValueError("at most 4 Kraus operators per channel")
        tab[i, : k.shape[0]] = k
        nk[i] = k.shape[0]
    return tab, nk


def brickwork(n: int, depth: int, seed: int, channel: np.ndarray, idle_noise: bool = False,
              name: str = "") -> Circuit:
    """Haar-random brickwork circuit; ``channel`` hits both qubits after every gate (and, if
    ``idle_noise``, also every qubit left idle by a layer)."""
    rng = np.random.default_rng(seed)
    max_pairs = n // 2
    gates = np.zeros((depth, max_pairs, 4, 4), dtype=np.complex128)
    events = np.full((depth, n), -1, dtype=np.int32)
    for l in range(depth):
        for i, q in enumerate(layer_pairs(n, l)):
            gates[l, i] = haar_unitary(rng, 4)
            events[l, q] = 0
            events[l, q + 1] = 0
        if idle_noise:
            events[l, :] = 0
    tab, nk = _pad_channels([channel])
    return Circuit(n=n, depth=depth, gates=gates, channels=tab, n_kraus=nk, events=events,
                   name=name)


@dataclasses.dataclass
class MixedCircuit:
    """Per-trajectory brickwork circuits over a shared gate pool (trajectories of different
    widths, depths, bond dimensions and noise strengths in one batch).  Arrays are padded to
    the widest trajectory n and the deepest one depth; trajectories are ordered so that
    equal (width, chi) are consecutive."""
    n: int
    depth: int
    gates: np.ndarray       # pool [n_gates][4][4] c128
    gate_id: np.ndarray     # [n_traj][depth][n // 2] int32, -1 = identity
    channels: np.ndarray    # [n_channels][4][2][2]
    n_kraus: np.ndarray
    events: np.ndarray      # [n_traj][depth][n] int32, -1 = none
    widths: np.ndarray      # [n_traj]
    depths: np.ndarray
    chis: np.ndarray
    name: str = ""

    @property
    def n_traj(self) -> int:
        return int(self.widths.shape[0])

    def trajectory_circuit(self, t: int) -> Circuit:
        """The uniform circuit of trajectory t on its own width and depth."""
        w, d = int(self.widths[t]), int(self.depths[t])
        gates = np.zeros((d, w // 2, 4, 4), dtype=np.complex128)
        for l in range(d):
            for i, q in enumerate(layer_pairs(w, l)):
                gates[l, i] = self.gates[self.gate_id[t, l, i]]
        ev = self.events[t, :d, :w].copy()
        used = sorted(set(int(x) for x in ev.ravel() if x >= 0))
        remap = {c: i for i, c in enumerate(used)}
        ev2 = np.vectorize(lambda x: remap.get(int(x), -1))(ev).astype(np.int32) if ev.size else ev
        tab = self.channels[used] if used else np.zeros((0, 4, 2, 2), dtype=np.complex128)
        nk = self.n_kraus[used] if used else np.zeros(0, dtype=np.int32)
        return Circuit(n=w, depth=d, gates=gates, channels=tab, n_kraus=nk, events=ev2, name=f"{self.name}[{t}]")


def mixed_brickwork(n_traj: int, seed: int, widths=(24, 64), depths=(16, 32), chis=(16, 32, 64, 128),
                    p_range=(0.005, 0.03), pool_size: int = 1 << 16, name: str = "") -> MixedCircuit:
    """Each trajectory its own Haar brickwork circuit: width ~ U{widths}, depth ~ U{depths},
    chi ~ U(chis), depolarizing p ~ U[p_range] on both qubits after every gate; gates are
    drawn by index from a pool of ``pool_size`` Haar gates.  Trajectories are sorted by
    (chi, width) so that equal shapes are consecutive."""
    rng = np.random.default_rng(seed)
    w = rng.integers(widths[0], widths[1] + 1, size=n_traj)
    d = rng.integers(depths[0], depths[1] + 1, size=n_traj)
    c = rng.choice(np.asarray(chis), size=n_traj)
    p = rng.uniform(p_range[0], p_range[1], size=n_traj)
    order = np.lexsort((w, c))
    w, d, c, p = w[order], d[order], c[order], p[order]
    pool = haar_unitaries(pool_size, seed + 1)
    nmax, dmax = int(w.max()), int(d.max())
    ids = rng.integers(0, pool_size, size=(n_traj, dmax, nmax // 2)).astype(np.int32)
    gate_id = np.full((n_traj, dmax, nmax // 2), -1, dtype=np.int32)
    events = np.full((n_traj, dmax, nmax), -1, dtype=np.int32)
    for l in range(dmax):
        par = l % 2
        slots = np.arange(nmax // 2)
        q_lo = par + 2 * slots
        for t in range(n_traj):
            if l >= d[t]:
                continue
            ok = q_lo + 1 < w[t]
            gate_id[t, l, slots[ok]] = ids[t, l, slots[ok]]
            events[t, l, q_lo[ok]] = t
            events[t, l, q_lo[ok] + 1] = t
    tab, nk = _pad_channels([depolarizing(float(x)) for x in p])
    return MixedCircuit(n=nmax, depth=dmax, gates=pool, gate_id=gate_id, channels=tab, n_kraus=nk,
                        events=events, widths=w.astype(np.int32), depths=d.astype(np.int32),
                        chis=c.astype(np.int32), name=name)


def config_mixed(n_traj: int = 16384) -> "MixedWorkload":
    """16384 trajectories, each its own circuit: width 24..64, depth 16..32, chi in
    {16, 32, 64, 128}, depolarizing p in [0.005, 0.03], gates from a pool of 2^16."""
    mc = mixed_brickwork(n_traj, seed=1003, name="mixed_w24-64_d16-32")
    return MixedWorkload(mc, seed=2003, name=f"mixed-w24-64-d16-32-chi16-128-{n_traj}traj")


@dataclasses.dataclass
class MixedWorkload:
    circuit: MixedCircuit
    seed: int
    name: str


def noiseless_copy(c: Circuit) -> Circuit:
    """Same gates, no noise events."""
    return dataclasses.replace(c, events=np.full_like(c.events, -1))


# ----------------------------------------------------------------------------- configs


@dataclasses.dataclass
class Workload:
    circuit: Circuit
    chi: int
    n_traj: int
    seed: int          # trajectory seed (branch sampling)
    name: str


def config_small_exact() -> Workload:
    """10-qubit chain, depth 10, depolarizing p=0.01 after each gate, chi=32 (exact),
    1000 trajectories."""
    c = brickwork(10, 10, seed=1001, channel=depolarizing(0.01), name="n10_d10_dep0.01")
    return Workload(c, chi=32, n_traj=1000, seed=2001, name="n10-d10-dep0.01-chi32-1000traj")


def config_ad_dephasing() -> Workload:
    """32-qubit chain, depth 20, amplitude damping 0.005 then dephasing 0.005 on every
    qubit in every layer, chi=64, 4096 trajectories."""
    ch = compose(amplitude_damping(0.005), dephasing(0.005))
    c = brickwork(32, 20, seed=1002, channel=ch, idle_noise=True, name="n32_d20_ad_df")
    return Workload(c, chi=64, n_traj=4096, seed=2002, name="n32-d20-ad0.005-df0.005-chi64-4096traj")


def config_wide(chi: int = 128, n_traj: int = 2048) -> Workload:
    """100-qubit chain, depth 40, depolarizing p=0.02 after each gate (the chi=128 and
    chi=256 workloads share this circuit)."""
    c = brickwork(100, 40, seed=1005, channel=depolarizing(0.02), name="n100_d40_dep0.02")
    return Workload(c, chi=chi, n_traj=n_traj, seed=2005,
                    name=f"n100-d40-dep0.02-chi{chi}-{n_traj}traj")


# ----------------------------------------------------------------------------- Lindbladians


@dataclasses.dataclass
class LindbladModel:
    """A time-independent Lindbladian on an open chain (Sec. "Time-independent Lindbladian
    systems"): H = sum_i h2 on (i, i+1) + sum_i h1 on i, and on every qubit the single-site
    jump operators ``jumps`` = [(c [2][2], rate gamma)]; Trotter step dt, ``steps`` steps (two
    brickwork layers each, every layer followed by the jump processes of every qubit for dt/2).

    The pair terms H_(i,i+1) = h2 + w_i h1 (x) I + w_(i+1) I (x) h1 sum to H: w = 1/2 for a
    site in two pairs, 1 for the two end sites (in one pair only)."""
    n: int
    dt: float
    steps: int
    h2: np.ndarray
    h1: np.ndarray
    jumps: list
    name: str = ""

    @property
    def depth(self) -> int:
        return 2 * self.steps

    def pair_hamiltonian(self, q: int) -> np.ndarray:
        wl = 1.0 if q == 0 else 0.5
        wr = 1.0 if q + 1 == self.n - 1 else 0.5
        return (np.asarray(self.h2, dtype=np.complex128) + wl * np.kron(self.h1, _I) + wr * np.kron(_I, self.h1))


def lindblad_circuit(model: LindbladModel, gates: dict, channel: np.ndarray, name: str = "") -> Circuit:
    """The brickwork circuit of a Trotterised model from its pair gates (dict q -> 4 x 4) and
    its jump channel (Kraus stack): layer l acts with gates[q] on the pairs of parity l % 2,
    then the channel hits every qubit (the idle end qubits included)."""
    n, depth = model.n, model.depth
    gt = np.zeros((depth, n // 2, 4, 4), dtype=np.complex128)
    for l in range(depth):
        for i, q in enumerate(layer_pairs(n, l)):
            gt[l, i] = gates[q]
    tab, nk = _pad_channels([np.asarray(channel, dtype=np.complex128)])
    events = np.zeros((depth, n), dtype=np.int32)
    return Circuit(n=n, depth=depth, gates=gt, channels=tab, n_kraus=nk, events=events,
                   name=name or model.name)


def amplitude_damping_rate(gamma_ad_per_layer: float, dt: float) -> float:
    """Jump rate gamma of c = |0><1| whose dt/2 jump process is amplitude damping with rate
    gamma_ad (the appendix on typical jump operators: gamma_AD = 1 - exp(-gamma tau))."""
    return -2.0 * np.log1p(-gamma_ad_per_layer) / dt


_SIGMA_MINUS = np.array([[0, 1], [0, 0]], dtype=np.complex128)


def lindblad_heisenberg(n: int = 16, steps: int = 300, dt: float = 0.01, gamma_ad: float = 0.002) -> LindbladModel:
    """The fixed Hamiltonian of the paper's first Lindbladian study: H = sum_i Y_i Y_(i+1) +
    0.35 X_i + 0.35 Y_i + 0.5 Z_i (open chain), amplitude damping of rate gamma_ad per layer."""
    return LindbladModel(n=n, dt=dt, steps=steps, h2=np.kron(_Y, _Y), h1=0.35 * _X + 0.35 * _Y + 0.5 * _Z,
                         jumps=[(_SIGMA_MINUS, amplitude_damping_rate(gamma_ad, dt))],
                         name=f"lindblad_heisenberg_n{n}_dt{dt}_ad{gamma_ad}")


def lindblad_random_ti(n: int = 12, steps: int = 300, dt: float = 0.01, gamma_ad: float = 0.002,
                       seed: int = 0) -> LindbladModel:
    """A random translation-invariant Lindbladian of the paper's second study: one random
    Hermitian 4 x 4 pair term (normally distributed real and imaginary parts, Hermitian part
    taken) repeated on every pair, amplitude damping of rate gamma_ad per layer."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    return LindbladModel(n=n, dt=dt, steps=steps, h2=0.5 * (g + g.conj().T), h1=np.zeros((2, 2), dtype=np.complex128),
                         jumps=[(_SIGMA_MINUS, amplitude_damping_rate(gamma_ad, dt))],
                         name=f"lindblad_random_ti_n{n}_dt{dt}_ad{gamma_ad}_s{seed}")


def random_two_site_states(count: int, chi_l: int, chi_r: int, seed: int,
                           dtype=np.complex64) -> np.ndarray:
    """``count`` complex Gaussian two-site tensors theta[a][s][t][b], each normalised to
    unit Frobenius norm (layout chi_l x 2 x 2 x chi_r)."""
    rng = np.random.default_rng(seed)
    shape = (count, chi_l, 2, 2, chi_r)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    x /= np.sqrt(np.sum(np.abs(x) ** 2, axis=(1, 2, 3, 4), keepdims=True))
    return x.astype(dtype)


def random_two_site_states_torch(count: int, chi_l: int, chi_r: int, seed: int, device: str = "cuda"):
    """Same distribution as ``random_two_site_states`` (complex64), drawn with torch's seeded
    generator directly on ``device``, for batches too large to draw on the host."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    shape = (count, chi_l, 2, 2, chi_r)
    x = torch.complex(torch.randn(shape, generator=g, device=device, dtype=torch.float32),
                      torch.randn(shape, generator=g, device=device, dtype=torch.float32))
    nrm = torch.linalg.vector_norm(x.reshape(count, -1), dim=1)
    x /= nrm.reshape(count, 1, 1, 1, 1)
    return x


def haar_unitaries(count: int, seed: int, d: int = 4) -> np.ndarray:
    """``count`` Haar-random d x d unitaries (batched form of ``haar_unitary``)."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((count, d, d)) + 1j * rng.standard_normal((count, d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    dg = np.diagonal(r, axis1=1, axis2=2)
    return (q * (dg / np.abs(dg))[:, None, :]).astype(np.complex128)


def random_mixing_params(count: int, seed: int, scale: float = 0.1) -> np.ndarray:
    """``count`` x 16 real parameters of a U(4) mixing, N(0, scale^2)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=(count, 16))


def random_density_matrices(count: int, seed: int, rank: Optional[int] = None) -> np.ndarray:
    """Random single-qubit density matrices (rank 1 or 2), for unravelling tests."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, 2, 2), dtype=np.complex128)
    for i in range(count):
        r = rank if rank is not None else 2
        g = rng.standard_normal((2, r)) + 1j * rng.standard_normal((2, r))
        m = g @ g.conj().T
        out[i] = m / np.trace(m).real
    return out
