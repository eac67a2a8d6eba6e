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
