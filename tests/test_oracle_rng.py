"""Pins of the counter-based generator and the branch-sampling rule."""
import numpy as np
import pytest

from oracle import rng


def test_splitmix64_published_vectors():
    # first outputs of SplitMix64 as published with its reference implementation
    assert rng.splitmix64_kth(0, 1) == 0xE220A8397B1DCDAF
    assert [rng.splitmix64_kth(1234567, k) for k in range(1, 6)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_uniform_range_and_keying():
    us = [rng.uniform(7, t, l, q) for t in range(4) for l in range(3) for q in range(5)]
    assert all(0.0 <= u < 1.0 for u in us)
    assert len(set(us)) == len(us)
    # the key is exactly output number 1 + (traj<<32 | layer<<16 | qubit)
    k = (3 << 32) | (2 << 16) | 4
    assert rng.uniform(7, 3, 2, 4) == (rng.splitmix64_kth(7, 1 + k) >> 11) * 2.0 ** -53
    with pytest.raises(ValueError):
        rng.event_key(1 << 31, 0, 0)


def test_uniform_is_uniform():
    us = np.array([rng.uniform(11, t, 0, 0) for t in range(20000)])
    assert abs(us.mean() - 0.5) < 0.01
    assert abs(us.var() - 1 / 12) < 0.005


def test_sample_branch_rules():
    p = [0.25, 0.0, 0.5, 0.25]
    assert rng.sample_branch(p, 0.0) == 0
    assert rng.sample_branch(p, 0.2499) == 0
    assert rng.sample_branch(p, 0.25) == 2      # zero-weight branch never chosen
    assert rng.sample_branch(p, 0.7499) == 2
    assert rng.sample_branch(p, 0.75) == 3
    assert rng.sample_branch([0.3, 0.7, 0.0], 0.9999999999999999) == 1
    # unnormalised weights are normalised by their sum
    assert rng.sample_branch([2.0, 2.0], 0.49) == 0
    assert rng.sample_branch([2.0, 2.0], 0.51) == 1
    with pytest.raises(ValueError):
        rng.sample_branch([0.0, 0.0], 0.5)
