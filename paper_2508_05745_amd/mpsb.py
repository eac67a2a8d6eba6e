"""ctypes binding of the mpsb HIP library (argument marshalling only).

Every step of the simulation runs in the library's HIP kernels; torch provides device
memory (uint8 / complex / float64 CUDA tensors) and the current stream.  There is no CPU
fallback: if the library is missing or no device is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpsb.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSUP, ENUM, EKRAUS = 0, -1, -2, -3, -4, -5, -6
FP32_BULK, FP64 = 0, 1
ORTHOGONAL, FIXED, HAAR_OPT, OPTIMAL, LEAST_UNITARY = 0, 1, 2, 3, 4
MAX_CHI = 256

_lib = None


class MpsbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mpsb error {code}: {msg}")
        self.code = code


class _Circuit(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("gates", ctypes.c_void_p), ("n_gates", ctypes.c_int),
                ("gate_id", ctypes.c_void_p), ("n_channels", ctypes.c_int),
                ("kraus", ctypes.c_void_p), ("n_kraus", ctypes.c_void_p), ("events", ctypes.c_void_p),
                ("events_per_traj", ctypes.c_int), ("unravel_mode", ctypes.c_int), ("fixed_u", ctypes.c_void_p)]


def lib():
    """Loads libmpsb.so (built in-tree by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is None:
        # torch (which brings its own HIP runtime) is imported before the library is loaded:
        # loaded the other way round, the library's runtime finds no device on the GPU machine
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build the HIP library first "
                               "(python -m paper_2508_05745_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t
        L.mps_last_error.restype = ctypes.c_char_p
        L.mps_batch_plan.argtypes = [i32, vp, vp, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.mps_batch_create.argtypes = [i32, vp, vp, i32, u64, ctypes.c_int64, vp, sz, vp, sz, vp, ctypes.POINTER(vp)]
        L.mps_batch_create_static.argtypes = [i32, vp, vp, i32, u64, ctypes.c_int64, vp, sz, vp, ctypes.POINTER(vp)]
        L.mps_circuit_bytes.argtypes = [vp, ctypes.POINTER(_Circuit), ctypes.POINTER(sz)]
        L.mps_batch_set_circuit.argtypes = [vp, ctypes.POINTER(_Circuit), vp, sz]
        L.mps_circuit_validate.argtypes = [i32, vp, ctypes.POINTER(_Circuit)]
        L.mps_batch_set_graphs.argtypes = [vp, i32]
        L.mps_batch_set_entropy.argtypes = [vp, vp]
        L.mps_batch_set_autotune.argtypes = [vp, i32]
        L.apply_layer.argtypes = [vp, i32, vp, vp, vp]
        L.apply_layer_replay.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.sample_kraus.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp]
        L.mps_truncate.argtypes = [vp, i32, vp]
        L.apply_layer_global.argtypes = [vp, i32, i32, vp]
        L.mps_sample_bitstrings.argtypes = [vp, i32, u64, vp]
        L.expect.argtypes = [vp, vp, vp, vp]
        L.mps_profile.argtypes = [vp, i32]
        L.mps_profile_read.argtypes = [vp, vp, vp, i32]
        L.mps_schedule_read.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32]
        L.mps_batch_sync.argtypes = [vp]
        L.mps_batch_destroy.argtypes = [vp]
        L.unravel_opt.argtypes = [i32, vp, vp, i32, vp, i32, vp, vp, vp, vp]
        L.mps_error_accumulate.argtypes = [i32, i32, vp, i32, ctypes.c_double, vp, vp]
        L.mps_error_estimate.argtypes = [i32, vp, ctypes.c_double, ctypes.c_double, vp, vp]
        L.mps_trotter_gate.argtypes = [vp, ctypes.c_double, vp]
        L.mps_jump_channel.argtypes = [i32, vp, vp, ctypes.c_double, vp, vp]
        L.unravel_cost.argtypes = [i32, vp, i32, i32, i32, vp, vp, vp, i32, vp, vp, vp]
        L.unravel_cost_grad.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, vp]
        L.unravel_cost_bond.argtypes = [i32, vp, i32, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp]
        L.unravel_cost_bond_grad.argtypes = [i32, vp, vp, vp, vp, vp, i32, vp, vp, vp]
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise MpsbError(code, lib().mps_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype).contiguous()


# ------------------------------------------------------------------------- circuits


class CircuitArrays:
    """Host arrays of a circuit in the layout the C ABI expects: an inputs.Circuit (one
    circuit shared by all trajectories), or an inputs.MixedCircuit (gate pool, per-trajectory
    gate ids and events)."""

    def __init__(self, circuit, mode: int = OPTIMAL, fixed_u: Optional[np.ndarray] = None):
        pooled = hasattr(circuit, "gate_id")
        self.n = circuit.n
        self.gates = np.ascontiguousarray(circuit.gates.astype(np.complex128)).view(np.float64)
        self.n_gates = circuit.gates.shape[0] if pooled else 0
        self.gate_id = np.ascontiguousarray(circuit.gate_id.astype(np.int32)) if pooled else None
        self.kraus = np.ascontiguousarray(circuit.channels.astype(np.complex128)).view(np.float64)
        self.n_kraus = np.ascontiguousarray(circuit.n_kraus.astype(np.int32))
        self.events = np.ascontiguousarray(circuit.events.astype(np.int32))
        self.events_per_traj = 1 if pooled else 0
        self.depth = circuit.depth
        self.mode = mode
        if fixed_u is not None:
            fx = np.asarray(fixed_u, dtype=np.complex128)
            fu = np.zeros((circuit.channels.shape[0], 4, 4), dtype=np.complex128)
            fu[..., :fx.shape[-1]] = fx           # 4 x r mixings are zero-padded to 4 x 4
            self.fixed_u = np.ascontiguousarray(fu).view(np.float64)
        else:
            self.fixed_u = None

    def struct(self) -> _Circuit:
        c = _Circuit()
        c.depth = self.depth
        c.gates = self.gates.ctypes.data
        c.n_gates = self.n_gates
        c.gate_id = self.gate_id.ctypes.data if self.gate_id is not None else None
        c.n_channels = self.n_kraus.shape[0]
        c.kraus = self.kraus.ctypes.data
        c.n_kraus = self.n_kraus.ctypes.data
        c.events = self.events.ctypes.data
        c.events_per_traj = self.events_per_traj
        c.unravel_mode = self.mode
        c.fixed_u = self.fixed_u.ctypes.data if self.fixed_u is not None else None
        return c


def _shape_arrays(n_traj: int, n_qubits, chi):
    w = np.ascontiguousarray(np.broadcast_to(np.asarray(n_qubits, dtype=np.int32), (n_traj,)))
    c = np.ascontiguousarray(np.broadcast_to(np.asarray(chi, dtype=np.int32), (n_traj,)))
    return w, c


def plan(n_traj: int, n_qubits, chi, precision: int):
    """(state_bytes, work_bytes); n_qubits and chi are ints or per-trajectory arrays."""
    w, c = _shape_arrays(n_traj, n_qubits, chi)
    s, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().mps_batch_plan(n_traj, w.ctypes.data, c.ctypes.data, precision, ctypes.byref(s),
                                ctypes.byref(wb)))
    return s.value, wb.value


def validate_circuit(circuit, mode: int = OPTIMAL, fixed_u=None, n_traj: int = 1, widths=None):
    ca = CircuitArrays(circuit, mode, fixed_u)
    st = ca.struct()
    w = np.ascontiguousarray(np.broadcast_to(np.asarray(circuit.n if widths is None else widths, dtype=np.int32),
                                             (n_traj,)))
    _check(lib().mps_circuit_validate(n_traj, w.ctypes.data, ctypes.byref(st)))


class Batch:
    """A batch of MPS trajectories living in caller (torch) device buffers.  n_qubits and
    chi are ints (uniform batch) or per-trajectory arrays (mixed batch: equal shapes must be
    consecutive).  Trajectory t draws its branches with the key traj_offset + t."""

    def __init__(self, n_traj: int, n_qubits, chi, precision: int = FP64, seed: int = 0,
                 traj_offset: int = 0, static_work: bool = False):
        """static_work: no work buffer is allocated; the batch runs on the library's static
        device work area (mps_batch_create_static: uniform batches of bounded size, one at a
        time per device)."""
        import torch
        self.widths, self.chis = _shape_arrays(n_traj, n_qubits, chi)
        self.n_traj, self.precision = n_traj, precision
        self.n = int(self.widths.max())
        self.chi = int(self.chis.max())
        self.mixed = bool((self.widths != self.widths[0]).any() or (self.chis != self.chis[0]).any())
        sb, wb = plan(n_traj, self.widths, self.chis, precision)
        self.state = torch.empty(sb, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        if static_work:
            self.work = None
            _check(lib().mps_batch_create_static(n_traj, self.widths.ctypes.data, self.chis.ctypes.data, precision,
                                                 ctypes.c_uint64(seed), ctypes.c_int64(traj_offset),
                                                 _ptr(self.state), sb, _stream(), ctypes.byref(h)))
        else:
            self.work = torch.empty(wb, dtype=torch.uint8, device="cuda")
            _check(lib().mps_batch_create(n_traj, self.widths.ctypes.data, self.chis.ctypes.data, precision,
                                          ctypes.c_uint64(seed), ctypes.c_int64(traj_offset), _ptr(self.state), sb,
                                          _ptr(self.work), wb, _stream(), ctypes.byref(h)))
        self.h = h
        self._circ = None
        self._cbuf = None

    def set_circuit(self, circuit, mode: int = OPTIMAL, fixed_u=None):
        import torch
        ca = CircuitArrays(circuit, mode, fixed_u)
        st = ca.struct()
        nb = ctypes.c_size_t()
        _check(lib().mps_circuit_bytes(self.h, ctypes.byref(st), ctypes.byref(nb)))
        buf = torch.empty(max(nb.value, 256), dtype=torch.uint8, device="cuda")
        _check(lib().mps_batch_set_circuit(self.h, ctypes.byref(st), _ptr(buf), nb.value))
        self._circ, self._cbuf = ca, buf

    def set_entropy(self, entropy=None):
        """Per-gate bond entropy output of the following layers: a float64 CUDA tensor
        [n_traj][W/2] (slot layout of `discarded`), or None to stop."""
        _check(lib().mps_batch_set_entropy(self.h, _ptr(entropy)))
        self._entropy = entropy

    def set_graphs(self, enable: bool):
        _check(lib().mps_batch_set_graphs(self.h, int(bool(enable))))

    def set_autotune(self, enable: bool):
        _check(lib().mps_batch_set_autotune(self.h, int(bool(enable))))

    def profile(self, mode: int):
        """0 off, 1 kernel classes, 2 member schedule, 3 both (resets the sums)."""
        _check(lib().mps_profile(self.h, int(mode)))

    def schedule_read(self):
        """Member schedule sums since profile(2|3): per member (first trajectory, trajectory
        count, stream, busy ms) as numpy arrays, then the summed layer wall time (ms) and the
        number of timed layers."""
        n = lib().mps_schedule_read(self.h, None, None, None, None, None, None, 0)
        _check(min(n, 0))
        first = np.zeros(n, dtype=np.int32)
        count = np.zeros(n, dtype=np.int32)
        stream = np.zeros(n, dtype=np.int32)
        busy = np.zeros(n, dtype=np.float64)
        el = ctypes.c_double()
        layers = ctypes.c_longlong()
        _check(min(0, lib().mps_schedule_read(self.h, first.ctypes.data, count.ctypes.data, stream.ctypes.data,
                                              busy.ctypes.data, ctypes.byref(el), ctypes.byref(layers), n)))
        return first, count, stream, busy, el.value, layers.value

    def apply_layer(self, layer: int, discarded=None, branch=None, w_record=None, w_in=None, branch_in=None):
        """w_in / branch_in (record layouts, device tensors): follow recorded mixings / branches."""
        if w_in is None and branch_in is None:
            _check(lib().apply_layer(self.h, layer, _ptr(discarded), _ptr(branch), _ptr(w_record)))
        else:
            _check(lib().apply_layer_replay(self.h, layer, _ptr(w_in), _ptr(branch_in), _ptr(discarded),
                                            _ptr(branch), _ptr(w_record)))

    def sample_kraus(self, qubit: int, channel: int, mode: int, rng_layer: int, forced=None,
                     branch=None, p=None):
        q = np.full(self.n_traj, qubit, dtype=np.int32)
        f = None if forced is None else np.ascontiguousarray(np.asarray(forced, dtype=np.int32))
        _check(lib().sample_kraus(self.h, q.ctypes.data, channel, mode, rng_layer,
                                  None if f is None else f.ctypes.data, _ptr(branch), _ptr(p)))

    def truncate(self, chi: int, discarded=None):
        _check(lib().mps_truncate(self.h, chi, _ptr(discarded)))

    def apply_layer_global(self, layer: int, chi: int, discarded=None):
        """Global layering: the layer without truncation below the capacities, then every
        bond truncated to chi (create the batch with capacity >= 2 chi)."""
        _check(lib().apply_layer_global(self.h, layer, chi, _ptr(discarded)))

    def sample_bitstrings(self, n_samples: int, seed: int):
        """uint8 CUDA tensor [n_traj][n_samples][n] of Born samples of every trajectory."""
        import torch
        bits = torch.empty((self.n_traj, n_samples, self.n), dtype=torch.uint8, device="cuda")
        _check(lib().mps_sample_bitstrings(self.h, n_samples, ctypes.c_uint64(seed), _ptr(bits)))
        return bits

    def expect(self, per_traj: bool = True):
        """(mean, m2, per_traj) of <Z_i> (n) then <Z_i Z_i+1> (n-1), float64 CUDA tensors
        (per_traj None unless asked for).  A mixed batch (widths up to W) uses the widest
        trajectory's layout: per_traj [n_traj][2W-1] NaN-padded rows, mean / m2 over the
        trajectories that have each observable (NaN where none has it)."""
        import torch
        nobs = 2 * self.n - 1
        pt = torch.empty((self.n_traj, nobs), dtype=torch.float64, device="cuda") if per_traj else None
        mean = torch.empty(nobs, dtype=torch.float64, device="cuda")
        m2 = torch.empty(nobs, dtype=torch.float64, device="cuda")
        _check(lib().expect(self.h, _ptr(mean), _ptr(m2), _ptr(pt)))
        return mean, m2, pt

    def sync(self):
        _check(lib().mps_batch_sync(self.h))

    def close(self):
        if self.h is not None:
            lib().mps_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------- Lindbladians


def trotter_gate(h, dt: float) -> np.ndarray:
    """exp(-i h dt) of a Hermitian 4 x 4 pair term (host, mps_trotter_gate)."""
    hh = np.ascontiguousarray(np.asarray(h, dtype=np.complex128))
    g = np.zeros((4, 4), dtype=np.complex128)
    _check(lib().mps_trotter_gate(hh.ctypes.data, ctypes.c_double(dt), g.ctypes.data))
    return g


def jump_channel(jumps, tau: float) -> np.ndarray:
    """Kraus operators [r][2][2] of the jump processes [(c, gamma)] of one site over time tau
    (host, mps_jump_channel)."""
    c = np.zeros((max(len(jumps), 1), 2, 2), dtype=np.complex128)
    g = np.zeros(max(len(jumps), 1))
    for i, (x, y) in enumerate(jumps):
        c[i], g[i] = np.asarray(x, dtype=np.complex128), float(y)
    k = np.zeros((4, 2, 2), dtype=np.complex128)
    r = ctypes.c_int()
    _check(lib().mps_jump_channel(len(jumps), c.ctypes.data, g.ctypes.data, ctypes.c_double(tau), k.ctypes.data,
                                  ctypes.byref(r)))
    return k[: r.value].copy()


def lindblad_circuit(model):
    """The model's Trotterised noisy brickwork circuit (inputs.LindbladModel), its gates and
    jump channel made by the library."""
    from . import inputs as I
    gates = {q: trotter_gate(model.pair_hamiltonian(q), model.dt) for q in range(model.n - 1)}
    return I.lindblad_circuit(model, gates, jump_channel(model.jumps, model.dt / 2))


# ------------------------------------------------------------------------- certified error

STEP_EXACT, STEP_PAPER = 0, 1


class ErrorBound:
    """Per-trajectory cumulated truncation error of a run (device FP64 accumulator) and the
    certified estimate of Thm. "Truncated Trajectory Sampling error"."""

    def __init__(self, n_traj: int, step_kind: int = STEP_EXACT):
        import torch
        self.n_traj, self.kind = n_traj, step_kind
        self.eps_tot = torch.zeros(n_traj, dtype=torch.float64, device="cuda")

    def add_layer(self, discarded, weight: float = 1.0):
        slots = discarded.shape[1]
        _check(lib().mps_error_accumulate(self.n_traj, slots, _ptr(discarded.contiguous()), self.kind,
                                          ctypes.c_double(weight), _ptr(self.eps_tot), _stream()))

    def estimate(self, eps_max: float = 4.0, delta: float = 0.05):
        """(eps_hat, Hoeffding buffer, bound) as host floats."""
        import torch
        out = torch.empty(3, dtype=torch.float64, device="cuda")
        _check(lib().mps_error_estimate(self.n_traj, _ptr(self.eps_tot), ctypes.c_double(eps_max),
                                        ctypes.c_double(delta), _ptr(out), _stream()))
        return tuple(float(x) for x in out.cpu())


# ------------------------------------------------------------------------- unravelling


def unravel_opt(rho_q, kraus, kraus_id=None):
    """Batched optimal unravelling.  rho_q: [B,2,2] complex; kraus: [n_k, r, 2, 2] (or
    [r,2,2]) complex.  Returns (U [B,4,r] complex128, p [B,4], eof [B]) CUDA tensors."""
    import torch
    rho = torch.as_tensor(rho_q).to(device="cuda", dtype=torch.complex128).contiguous()
    k = torch.as_tensor(kraus).to(device="cuda", dtype=torch.complex128)
    if k.dim() == 3:
        k = k.unsqueeze(0)
    k = k.contiguous()
    B, nk, r = rho.shape[0], k.shape[0], k.shape[1]
    kid = None if kraus_id is None else torch.as_tensor(kraus_id).to(device="cuda", dtype=torch.int32).contiguous()
    U = torch.empty((B, 4, r), dtype=torch.complex128, device="cuda")
    p = torch.empty((B, 4), dtype=torch.float64, device="cuda")
    eof = torch.empty((B,), dtype=torch.float64, device="cuda")
    _check(lib().unravel_opt(B, _ptr(rho), _ptr(k), nk, _ptr(kid), r, _ptr(U), _ptr(p),
                             _ptr(eof), _stream()))
    return U, p, eof


def unravel_cost(theta, kraus, params, u_ref, kind: int = 0):
    """theta: [B, chi_l, 2, 2, chi_r] complex64/complex128 CUDA tensor.  Returns (f [B],
    rho_q [B,2,2])."""
    import torch
    prec = FP32_BULK if theta.dtype == torch.complex64 else FP64
    B, cl, cr = theta.shape[0], theta.shape[1], theta.shape[4]
    k = torch.zeros((4, 2, 2), dtype=torch.complex128, device="cuda")
    kk = torch.as_tensor(kraus).to(device="cuda", dtype=torch.complex128)
    k[: kk.shape[0]] = kk
    f = torch.empty((B,), dtype=torch.float64, device="cuda")
    rho = torch.empty((B, 2, 2), dtype=torch.complex128, device="cuda")
    params = params.contiguous()
    u_ref = u_ref.to(torch.complex128).contiguous()
    _check(lib().unravel_cost(B, _ptr(theta.contiguous()), cl, cr, prec, _ptr(k), _ptr(params),
                              _ptr(u_ref), kind, _ptr(f), _ptr(rho), _stream()))
    return f, rho, k


def unravel_cost_grad(rho, kraus4, params, u_ref, kind: int, grad_f):
    import torch
    B = rho.shape[0]
    g = torch.empty((B, 16), dtype=torch.float64, device="cuda")
    _check(lib().unravel_cost_grad(B, _ptr(rho.contiguous()), _ptr(kraus4.contiguous()),
                                   _ptr(params.contiguous()), _ptr(u_ref.contiguous()), kind,
                                   _ptr(None if grad_f is None else grad_f.contiguous()),
                                   _ptr(g), _stream()))
    return g


def unravel_cost_bond(theta, kraus, params, u_ref, kind: int = 0):
    """The cost across the block's internal bond.  theta: [B, chi_l, 2, 2, chi_r] complex64 /
    complex128 CUDA tensor.  Returns (f [B], rho_q [B,2,2], N [B,4,4], kraus padded to 4)."""
    import torch
    prec = FP32_BULK if theta.dtype == torch.complex64 else FP64
    B, cl, cr = theta.shape[0], theta.shape[1], theta.shape[4]
    k = torch.zeros((4, 2, 2), dtype=torch.complex128, device="cuda")
    kk = torch.as_tensor(kraus).to(device="cuda", dtype=torch.complex128)
    k[: kk.shape[0]] = kk
    f = torch.empty((B,), dtype=torch.float64, device="cuda")
    rho = torch.empty((B, 2, 2), dtype=torch.complex128, device="cuda")
    nm = torch.empty((B, 4, 4), dtype=torch.complex128, device="cuda")
    params = params.contiguous()
    u_ref = u_ref.to(torch.complex128).contiguous()
    _check(lib().unravel_cost_bond(B, _ptr(theta.contiguous()), cl, cr, prec, _ptr(k), _ptr(params),
                                   _ptr(u_ref), kind, _ptr(f), _ptr(rho), _ptr(nm), _stream()))
    return f, rho, nm, k


def unravel_cost_bond_grad(rho, nm, kraus4, params, u_ref, kind: int, grad_f):
    import torch
    B = rho.shape[0]
    g = torch.empty((B, 16), dtype=torch.float64, device="cuda")
    _check(lib().unravel_cost_bond_grad(B, _ptr(rho.contiguous()), _ptr(nm.contiguous()),
                                        _ptr(kraus4.contiguous()), _ptr(params.contiguous()),
                                        _ptr(u_ref.contiguous()), kind,
                                        _ptr(None if grad_f is None else grad_f.contiguous()),
                                        _ptr(g), _stream()))
    return g


def _autograd_function(bond: bool):
    import torch

    class UnravelCost(torch.autograd.Function):
        """f(params) = expected linear (kind 0) / Renyi-2 (kind 1) entropy of the unravelling
        of `kraus` on the states `theta` (between the noisy qubit and the rest of the block,
        or across the block's internal bond); differentiable w.r.t. params only (the adjoint
        is the library's unravel_cost_grad / unravel_cost_bond_grad, theta is not re-read)."""

        @staticmethod
        def forward(ctx, params, theta, kraus, u_ref, kind):
            if bond:
                f, rho, nm, k4 = unravel_cost_bond(theta, kraus, params, u_ref, kind)
            else:
                f, rho, k4 = unravel_cost(theta, kraus, params, u_ref, kind)
                nm = rho
            ctx.save_for_backward(rho, nm, k4, params, u_ref.to(torch.complex128))
            ctx.kind = kind
            return f

        @staticmethod
        def backward(ctx, grad_f):
            rho, nm, k4, params, u_ref = ctx.saved_tensors
            gf = grad_f.to(torch.float64)
            if bond:
                g = unravel_cost_bond_grad(rho, nm, k4, params, u_ref, ctx.kind, gf)
            else:
                g = unravel_cost_grad(rho, k4, params, u_ref, ctx.kind, gf)
            return g, None, None, None, None

    return UnravelCost


_UC = {}


def UnravelCost(bond: bool = False):
    if bond not in _UC:
        _UC[bond] = _autograd_function(bond)
    return _UC[bond]
