"""The C-ABI library loads, exports every entry point declared in include/mpsb.h, and
validates its arguments on the host (no GPU calls)."""
import os
import re

import numpy as np
import pytest

from paper_2508_05745_amd import inputs as I
from paper_2508_05745_amd import mpsb as M

HDR = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "mpsb.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = M.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n


def test_plan_sizes_and_errors():
    s1, w1 = M.plan(16, 10, 32, M.FP64)
    s2, w2 = M.plan(16, 10, 32, M.FP32_BULK)
    assert s1 == 2 * s2 and s1 > 0 and w1 > 0
    # bond capacities min(chi, 2^(k+1), 2^(n-k-1)): n=10, chi=32 -> 2,4,8,16,32,16,8,4,2
    caps = [2, 4, 8, 16, 32, 16, 8, 4, 2]
    dl = [1] + caps
    dr = caps + [1]
    elems = sum((2 * a * b + 31) // 32 * 32 for a, b in zip(dl, dr))
    assert s1 == 16 * elems * 16
    for args in [(0, 10, 32, 1), (4, 1, 32, 1), (4, 10, 0, 1), (4, 10, 257, 1), (4, 10, 8, 7)]:
        with pytest.raises(M.MpsbError) as e:
            M.plan(*args)
        assert e.value.code == M.EINVAL


def test_circuit_validation():
    c = I.brickwork(6, 3, seed=1, channel=I.depolarizing(0.1))
    M.validate_circuit(c)
    bad = I.brickwork(6, 3, seed=1, channel=I.depolarizing(0.1))
    bad.channels = bad.channels.copy()
    bad.channels[0, 0] *= 1.01                       # not trace preserving
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(bad)
    assert e.value.code == M.EKRAUS
    bad2 = I.brickwork(6, 3, seed=1, channel=I.depolarizing(0.1))
    bad2.gates = bad2.gates.copy()
    bad2.gates[1, 0] *= 1.001                        # not unitary
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(bad2)
    assert e.value.code == M.EINVAL
    bad3 = I.brickwork(6, 3, seed=1, channel=I.depolarizing(0.1))
    bad3.events = bad3.events.copy()
    bad3.events[0, 0] = 3                            # no such channel
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(bad3)
    assert e.value.code == M.EINVAL
    bad4 = I.brickwork(6, 3, seed=1, channel=I.depolarizing(0.1))
    bad4.gates = bad4.gates.copy()
    bad4.gates[0, 0, 0, 0] = np.nan
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(bad4)
    assert e.value.code == M.ENUM
    # FIXED mixings must be isometries on the used columns
    with pytest.raises(M.MpsbError):
        M.validate_circuit(c, M.FIXED, 2 * np.eye(4))
    M.validate_circuit(c, M.FIXED, np.eye(4))
    # named unravelings: Haar Optimal needs 1, 2 or 4 Kraus operators per channel
    M.validate_circuit(c, M.HAAR_OPT)
    M.validate_circuit(c, M.LEAST_UNITARY)
    three = I.brickwork(6, 3, seed=1, channel=I.dephasing(0.1))
    three.channels = np.zeros((1, 4, 2, 2), dtype=np.complex128)
    p = 0.1
    three.channels[0, :3] = [np.sqrt(1 - p) * np.eye(2), np.sqrt(p) * np.diag([1.0, 0.0]), np.sqrt(p) * np.diag([0.0, 1.0])]
    three.n_kraus = np.array([3])
    M.validate_circuit(three, M.OPTIMAL)
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(three, M.HAAR_OPT)
    assert e.value.code == M.EINVAL
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(c, 5)
    assert e.value.code == M.EINVAL


def test_mixed_plan_is_the_sum_of_its_runs():
    w = np.array([10, 10, 12, 12, 12, 12], dtype=np.int32)
    c = np.array([8, 8, 8, 8, 16, 16], dtype=np.int32)
    s, wb = M.plan(6, w, c, M.FP32_BULK)
    parts = [M.plan(2, 10, 8, M.FP32_BULK), M.plan(2, 12, 8, M.FP32_BULK), M.plan(2, 12, 16, M.FP32_BULK)]
    al = lambda x: (x + 255) // 256 * 256
    assert s == sum(al(p[0]) for p in parts) and wb == sum(al(p[1]) for p in parts)
    # a uniform batch given as arrays plans exactly as the scalar form
    assert M.plan(5, np.full(5, 10), np.full(5, 8), M.FP64) == M.plan(5, 10, 8, M.FP64)


def test_pooled_circuit_validation():
    mc = I.mixed_brickwork(12, seed=7, widths=(6, 9), depths=(3, 5), chis=(4, 8), pool_size=32)
    M.validate_circuit(mc, n_traj=mc.n_traj, widths=mc.widths)
    bad = I.MixedCircuit(**{**mc.__dict__, "gate_id": mc.gate_id.copy()})
    bad.gate_id[0, 0, 0] = 32
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(bad, n_traj=mc.n_traj, widths=mc.widths)
    assert e.value.code == M.EINVAL
    bad2 = I.MixedCircuit(**{**mc.__dict__, "gates": mc.gates.copy()})
    bad2.gates[3] *= 1.01
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(bad2, n_traj=mc.n_traj, widths=mc.widths)
    assert e.value.code == M.EINVAL
    bad3 = I.MixedCircuit(**{**mc.__dict__, "events": mc.events.copy()})
    bad3.events[2, 1, 0] = mc.channels.shape[0]
    with pytest.raises(M.MpsbError) as e:
        M.validate_circuit(bad3, n_traj=mc.n_traj, widths=mc.widths)
    assert e.value.code == M.EINVAL


def test_mixed_trajectory_circuit_matches_the_tables():
    mc = I.mixed_brickwork(8, seed=3, widths=(5, 9), depths=(2, 4), chis=(4,), pool_size=16)
    for t in range(mc.n_traj):
        c = mc.trajectory_circuit(t)
        assert c.n == mc.widths[t] and c.depth == mc.depths[t]
        for l in range(c.depth):
            for i, q in enumerate(c.pairs(l)):
                assert np.array_equal(c.gates[l, i], mc.gates[mc.gate_id[t, l, i]])
                assert c.events[l, q] >= 0 and c.events[l, q + 1] >= 0
        # past the trajectory's width / depth: identity and no events
        assert (mc.gate_id[t, c.depth:] == -1).all() and (mc.events[t, c.depth:] == -1).all()
        assert (mc.events[t, :, c.n:] == -1).all()


def test_unravel_entry_points_validate_on_the_host():
    """Sizes and the channel count are checked before any device work (no GPU needed: the
    calls fail on the host with null device pointers never dereferenced)."""
    import ctypes
    lib = M.lib()
    one = ctypes.c_void_p(8)   # never dereferenced: validation fails first
    assert lib.unravel_opt(-1, one, one, 1, None, 2, one, one, one, None) == M.EINVAL
    assert lib.unravel_opt(4, one, one, 0, None, 2, one, one, one, None) == M.EINVAL
    assert lib.unravel_opt(4, one, one, 1, None, 5, one, one, one, None) == M.EINVAL
    assert lib.unravel_opt(4, None, one, 1, None, 2, one, one, one, None) == M.EINVAL
    assert lib.unravel_opt(0, None, None, 1, None, 2, None, None, None, None) == M.OK
    assert lib.unravel_cost(4, one, 8, 8, 3, one, one, one, 0, one, one, None) == M.EINVAL
    assert lib.unravel_cost(4, one, 8, 8, 0, one, one, one, 2, one, one, None) == M.EINVAL
    assert lib.unravel_cost_grad(4, one, one, one, one, 5, None, one, None) == M.EINVAL
    assert lib.unravel_cost_grad(4, None, one, one, one, 0, None, one, None) == M.EINVAL
    assert lib.unravel_cost_bond(4, one, 8, 8, 3, one, one, one, 0, one, one, one, None) == M.EINVAL
    assert lib.unravel_cost_bond(4, one, 8, 8, 1, one, one, one, 2, one, one, one, None) == M.EINVAL
    assert lib.unravel_cost_bond(4, one, 0, 8, 1, one, one, one, 0, one, one, one, None) == M.EINVAL
    assert lib.unravel_cost_bond(4, one, 1 << 14, 1 << 13, 1, one, one, one, 0, one, one, one, None) == M.EINVAL
    assert lib.unravel_cost_bond(4, one, 8, 8, 1, one, one, one, 0, one, one, None, None) == M.EINVAL
    assert lib.unravel_cost_bond(0, None, 8, 8, 1, None, None, None, 0, None, None, None, None) == M.OK
    assert lib.unravel_cost_bond_grad(4, one, None, one, one, one, 0, None, one, None) == M.EINVAL
    assert lib.unravel_cost_bond_grad(4, one, one, one, one, one, 3, None, one, None) == M.EINVAL
    big = (1 << 26) + 1   # above MPSB_MAX_COST_BATCH
    assert lib.unravel_cost(big, one, 1, 1, 1, one, one, one, 0, one, one, None) == M.EINVAL
    assert lib.unravel_cost_grad(big, one, one, one, one, 0, None, one, None) == M.EINVAL
    assert lib.unravel_cost_bond(big, one, 1, 1, 1, one, one, one, 0, one, one, one, None) == M.EINVAL
    assert lib.unravel_cost_bond_grad(big, one, one, one, one, one, 0, None, one, None) == M.EINVAL


def test_static_batch_rejects_oversized_and_mixed_plans():
    """mps_batch_create_static checks the planned work memory against the static area and
    rejects mixed batches before touching any device."""
    import ctypes
    lib = M.lib()
    h = ctypes.c_void_p()
    one = ctypes.c_void_p(256)
    w = np.full(2048, 100, dtype=np.int32)
    c = np.full(2048, 128, dtype=np.int32)
    _, wb = M.plan(2048, 100, 128, M.FP64)
    assert wb > (64 << 20)
    r = lib.mps_batch_create_static(2048, w.ctypes.data, c.ctypes.data, M.FP64, 1, 0, one, 1 << 40, None, ctypes.byref(h))
    assert r == M.ENOMEM and b"static work area" in lib.mps_last_error()
    w2 = np.array([6, 6, 8], dtype=np.int32)
    c2 = np.array([4, 4, 4], dtype=np.int32)
    r = lib.mps_batch_create_static(3, w2.ctypes.data, c2.ctypes.data, M.FP64, 1, 0, one, 1 << 40, None, ctypes.byref(h))
    assert r == M.ENOTSUP


def test_error_entry_points_validate_on_the_host():
    import ctypes
    lib = M.lib()
    one = ctypes.c_void_p(256)
    assert lib.mps_error_accumulate(4, 2, one, 2, ctypes.c_double(1.0), one, None) == M.EINVAL
    assert lib.mps_error_accumulate(4, 2, one, 0, ctypes.c_double(-1.0), one, None) == M.EINVAL
    assert lib.mps_error_accumulate(4, 2, None, 0, ctypes.c_double(1.0), one, None) == M.EINVAL
    assert lib.mps_error_accumulate(0, 2, None, 0, ctypes.c_double(1.0), None, None) == M.OK
    assert lib.mps_error_estimate(4, one, ctypes.c_double(1.5), ctypes.c_double(0.05), one, None) == M.EINVAL
    assert lib.mps_error_estimate(4, one, ctypes.c_double(4.0), ctypes.c_double(1.0), one, None) == M.EINVAL
    assert lib.mps_error_estimate(0, one, ctypes.c_double(4.0), ctypes.c_double(0.05), one, None) == M.EINVAL


def test_lindblad_constructors_validate_on_the_host():
    """Error paths of the host-side Lindbladian constructors (no device involved)."""
    g = np.zeros((4, 4), dtype=np.complex128)
    g[0, 1] = 1.0                                     # not Hermitian
    with pytest.raises(M.MpsbError) as e:
        M.trotter_gate(g, 0.1)
    assert e.value.code == M.EINVAL
    g[0, 1] = np.nan
    with pytest.raises(M.MpsbError) as e:
        M.trotter_gate(g, 0.1)
    assert e.value.code == M.ENUM
    sm = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    with pytest.raises(M.MpsbError) as e:
        M.jump_channel([(sm, -1.0)], 0.1)
    assert e.value.code == M.EINVAL
    with pytest.raises(M.MpsbError) as e:
        M.jump_channel([(sm, 1.0)], -0.1)
    assert e.value.code == M.EINVAL
    with pytest.raises(M.MpsbError) as e:
        M.jump_channel([], 0.1)


def test_profile_and_schedule_read_validate_on_the_host():
    """Null handles are rejected before any device work (the handle-level checks that need a
    device are in the GPU schedule test)."""
    lib = M.lib()
    assert lib.mps_profile(None, 2) == M.EINVAL
    assert lib.mps_profile_read(None, None, None, 0) == M.EINVAL
    assert lib.mps_schedule_read(None, None, None, None, None, None, None, 0) == M.EINVAL
