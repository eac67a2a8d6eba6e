"""The entry point that allocates nothing (mps_batch_create_static: the batch's work memory is
the library's static device area) against the ordinary one (mps_batch_create with a caller
work buffer): the same kernels on the same inputs give the same per-trajectory observables
and branch records, bit for bit, on two batches in a row, the second smaller (the area keeps
the first batch's contents, which the second must not see)."""
import numpy as np
import pytest

from paper_2508_05745_amd import inputs as I

pytestmark = pytest.mark.gpu


def _run(c, chi, n_traj, prec, seed, static):
    import torch

    from paper_2508_05745_amd import mpsb as M
    b = M.Batch(n_traj, c.n, chi, prec, seed, static_work=static)
    b.set_circuit(c, M.OPTIMAL)
    b.set_graphs(False)
    br = torch.zeros((n_traj, c.n), dtype=torch.int32, device="cuda")
    d = torch.zeros((n_traj, c.n // 2), dtype=torch.float64, device="cuda")
    brs, ds = [], []
    for l in range(c.depth):
        b.apply_layer(l, discarded=d, branch=br)
        brs.append(br.cpu().numpy().copy())
        ds.append(d.cpu().numpy().copy())
    mean, m2, pt = b.expect()
    b.sync()
    out = dict(pt=pt.cpu().numpy(), mean=mean.cpu().numpy(), br=np.stack(brs), d=np.stack(ds))
    b.close()
    return out


@pytest.mark.parametrize("prec", [1, 0])
def test_static_work_matches_caller_work(prec):
    from paper_2508_05745_amd import mpsb as M
    cases = [(I.brickwork(12, 8, seed=61, channel=I.depolarizing(0.03)), 16, 96, 71),
             (I.brickwork(9, 6, seed=62, channel=I.compose(I.amplitude_damping(0.05), I.dephasing(0.05)),
                          idle_noise=True), 8, 40, 72)]
    for c, chi, n_traj, seed in cases:
        _, wb = M.plan(n_traj, c.n, chi, prec)
        assert wb <= (64 << 20)
        ref = _run(c, chi, n_traj, prec, seed, False)
        got = _run(c, chi, n_traj, prec, seed, True)
        for k in ("br", "d", "pt", "mean"):
            assert np.array_equal(got[k], ref[k]), (k, c.n, n_traj)
        assert np.isfinite(got["pt"]).all()


def test_static_work_is_held_by_one_batch_and_bounded():
    from paper_2508_05745_amd import mpsb as M
    a = M.Batch(4, 6, 4, M.FP64, 1, static_work=True)
    with pytest.raises(M.MpsbError) as e:
        M.Batch(4, 6, 4, M.FP64, 1, static_work=True)
    assert e.value.code == M.ENOTSUP
    with pytest.raises(M.MpsbError) as e:
        a.set_graphs(True)
    assert e.value.code == M.ENOTSUP
    a.close()
    b = M.Batch(4, 6, 4, M.FP64, 1, static_work=True)   # released by the first batch's destroy
    b.close()
