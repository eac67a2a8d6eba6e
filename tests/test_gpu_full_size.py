"""Parity at the full sizes of the workloads, in the launch configuration of a production
run (every trajectory of the batch in each launch, full bond capacities), checked on
sampled trajectories that the oracle replays one by one (recorded optimal mixings, checked
for completeness and optimality; branch choices and observables must match), plus
properties that hold at any size (FP32-bulk and FP64 trajectory averages agree
statistically).

Workloads: the 32-qubit amplitude-damping + dephasing circuit (depth 20, chi 64, 4096
trajectories, noise on every qubit in every layer), the 100-qubit depolarizing circuit at
chi 128 with 2048 trajectories over the layers the benchmark times (1 warm-up + 2), 20-qubit
circuits whose middle bonds saturate chi = 128 and chi = 256, and the chi = 256 case of the
100-qubit circuit (FP32-bulk with 2048 trajectories; FP64 in a memory wave of 1024).

Tolerances are flat: 1e-10 per observable of every replayed FP64 trajectory, 1e-4 for
FP32-bulk."""
import numpy as np
import pytest

from paper_2508_05745_amd import inputs as I

from gpu_util import replay_sampled, run_gpu_sampled

pytestmark = pytest.mark.gpu

# precision -> (per-trajectory observable tolerance, optimality gap of the recorded mixings)
TOL = {1: (1e-10, 1e-9), 0: (1e-4, 1e-4)}


def _check_replays(c, chi, seed, out, prec, tag):
    """Per-trajectory tolerance, flat: 1e-10 (FP64) / 1e-4 (FP32-bulk) on every observable
    of every replayed trajectory, truncating layers included."""
    tol, gap = TOL[prec]
    for row, t in enumerate(out["sample"]):
        ref, rp, js_gpu, js_ref, spectra = replay_sampled(c, chi, seed, out, row)
        assert js_gpu == js_ref, (tag, t)
        assert rp.max_incomplete < 1e-10, (tag, t, rp.max_incomplete)
        assert rp.max_gap < gap, (tag, t, rp.max_gap)
        err = np.abs(out["per_traj"][row] - ref).max()
        ncut = sum(1 for s in spectra if min(chi, s.size) < s.size and s[min(chi, s.size)] > 1e-12 * s[0])
        print(f"{tag} traj {t}: max |d<O>| = {err:.2e} over {len(spectra)} splits ({ncut} truncating), "
              f"optimality gap {rp.max_gap:.1e}", flush=True)
        assert err < tol, (tag, t, err, tol)


def _check_statistics(a, b, n_traj, zmax=4.5):
    se = np.sqrt(a["m2"] / (n_traj - 1) / n_traj + b["m2"] / (n_traj - 1) / n_traj) + 1e-15
    z = np.abs(a["mean"] - b["mean"]) / se
    print(f"FP32-bulk vs FP64 averages: max |d mean| {np.abs(a['mean'] - b['mean']).max():.2e}, max z {z.max():.2f}",
          flush=True)
    assert z.max() < zmax


def test_ad_dephasing_full_size():
    wl = I.config_ad_dephasing()
    c = wl.circuit
    sample = [0, 2049, wl.n_traj - 1]
    print(f"workload {wl.name}", flush=True)
    a = run_gpu_sampled(c, wl.chi, wl.n_traj, wl.seed, 1, 3, c.depth, sample)
    _check_replays(c, wl.chi, wl.seed, a, 1, "fp64")
    b = run_gpu_sampled(c, wl.chi, wl.n_traj, wl.seed, 0, 3, c.depth, sample[:1])
    _check_replays(c, wl.chi, wl.seed, b, 0, "fp32")
    _check_statistics(a, b, wl.n_traj)


def test_benchmark_workload_chi128_timed_layers():
    wl = I.config_wide(chi=128, n_traj=2048)
    c = wl.circuit
    sample = [0, 1024, wl.n_traj - 1]
    print(f"workload {wl.name}, layers 0-2", flush=True)
    a = run_gpu_sampled(c, wl.chi, wl.n_traj, wl.seed, 1, 3, 3, sample)
    _check_replays(c, wl.chi, wl.seed, a, 1, "fp64")
    b = run_gpu_sampled(c, wl.chi, wl.n_traj, wl.seed, 0, 3, 3, sample)
    _check_replays(c, wl.chi, wl.seed, b, 0, "fp32")
    _check_statistics(a, b, wl.n_traj)


def test_benchmark_workload_saturated_fp32_vs_fp64():
    """The benchmark's timed layers with saturated bonds (layers 0-9, chi = 128 reached at
    layer 7): the FP32-bulk and FP64 trajectory averages of all 199 observables agree within
    their combined statistical error (independent optimal unravellings of the same channel
    give the same average state)."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    wl = I.config_wide(chi=128, n_traj=2048)
    c = wl.circuit
    res = {}
    for prec in (1, 0):
        b = M.Batch(wl.n_traj, c.n, wl.chi, prec, wl.seed)
        b.set_circuit(c, M.OPTIMAL)
        for l in range(10):
            b.apply_layer(l)
        mean, m2, _ = b.expect(per_traj=False)
        b.sync()
        res[prec] = dict(mean=mean.cpu().numpy(), m2=m2.cpu().numpy())
        b.close()
        torch.cuda.empty_cache()
        print(f"precision {prec} done", flush=True)
    _check_statistics(res[1], res[0], wl.n_traj)


@pytest.mark.parametrize("prec", [1, 0])
def test_saturated_chi128(prec):
    """20 qubits, depth 12: the middle bonds reach and are truncated at chi = 128, so the
    bulk-bond kernels (m = 256 eigensolver, large theta tiles) run on saturated tensors."""
    c = I.brickwork(20, 12, seed=1006, channel=I.depolarizing(0.02))
    out = run_gpu_sampled(c, 128, 256, 2006, prec, 3, c.depth, [0, 255])
    _check_replays(c, 128, 2006, out, prec, f"prec{prec}")


@pytest.mark.parametrize("prec", [1, 0])
def test_saturated_chi24(prec):
    """Bond capacity 24, not a multiple of the 16-wide MFMA tiles: the centre hops (n = 24,
    24 x 48 and 48 x 24 centre tensors), the truncation Grams (m = 48) and the theta tiles all
    run on partial tiles once the middle bonds saturate."""
    c = I.brickwork(12, 10, seed=1024, channel=I.depolarizing(0.02))
    out = run_gpu_sampled(c, 24, 64, 2024, prec, 3, c.depth, [0, 63])
    _check_replays(c, 24, 2024, out, prec, f"chi24 prec{prec}")


@pytest.mark.parametrize("prec", [1, 0])
def test_saturated_chi256(prec):
    """20 qubits, depth 12: the middle bonds (capacity 256) reach and are truncated at
    chi = 256 in the last layers, so the m = 512 eigensolver instances (tridiagonalisation,
    back-transformation panels) and the centre hops of bonds above 128 run on dense spectra."""
    c = I.brickwork(20, 12, seed=1007, channel=I.depolarizing(0.02))
    out = run_gpu_sampled(c, 256, 128, 2007, prec, 3, c.depth, [0, 127])
    _check_replays(c, 256, 2007, out, prec, f"chi256 prec{prec}")


@pytest.mark.parametrize("prec,n_traj", [(0, 2048), (1, 1024)])
def test_wide_chi256_first_layer(prec, n_traj):
    wl = I.config_wide(chi=256, n_traj=n_traj)
    c = wl.circuit
    out = run_gpu_sampled(c, 256, n_traj, wl.seed, prec, 3, 1, [0, n_traj - 1])
    _check_replays(c, 256, wl.seed, out, prec, f"chi256 prec{prec}")


def test_unravel_cost_full_size():
    """65536 normalised complex-Gaussian two-site states (chi 64 on each side, c64, drawn on
    the device), 4-Kraus depolarizing p = 0.02, mixing parameters N(0, 0.1^2) around Haar
    reference unitaries: linear and Renyi-2 cost and adjoint gradient for the whole batch in
    one call; 1024 (256 for Renyi-2) spread states against the oracle's reduced state, cost
    and torch-CPU gradient, 256 (64) against central finite differences; and, on 1024
    states at their Wootters mixings (parameters 0), f = C^2 / 2 with a vanishing gradient."""
    import torch

    from oracle import cost as CO
    from oracle import unravel as OU
    from paper_2508_05745_amd import mpsb as M
    B = 65536
    th = I.random_two_site_states_torch(B, 64, 64, seed=4004)
    params = I.random_mixing_params(B, seed=4005)
    uref = I.haar_unitaries(B, seed=4006)
    k = I.depolarizing(0.02)
    pp = torch.as_tensor(params).cuda()
    uu = torch.as_tensor(uref).cuda()
    sample = np.linspace(0, B - 1, 1024).astype(np.int64)
    sidx = torch.as_tensor(sample).cuda()
    ths = th[sidx].cpu().numpy().astype(np.complex128)
    for kind, n_ref, n_fd in ((0, 1024, 256), (1, 256, 64)):
        f, rho, k4 = M.unravel_cost(th, k, pp, uu, kind)
        g = M.unravel_cost_grad(rho, k4, pp, uu, kind, None)
        f, rho, g = f.cpu().numpy(), rho.cpu().numpy(), g.cpu().numpy()
        assert np.isfinite(f).all() and np.isfinite(g).all()
        worst = [0.0, 0.0, 0.0, 0.0]
        for i, b in enumerate(sample[:n_ref]):
            r_ref = CO.rho_from_theta(ths[i])
            rn = r_ref / np.trace(r_ref).real
            f_ref, g_ref = CO.grad_torch(rn, k, params[b], uref[b], kind)
            worst[0] = max(worst[0], np.abs(rho[b] - r_ref).max())
            worst[1] = max(worst[1], abs(f[b] - f_ref))
            worst[2] = max(worst[2], np.linalg.norm(g[b] - g_ref) / max(1.0, np.linalg.norm(g_ref)))
            if i < n_fd:
                gfd = CO.grad_fd(rn, k, params[b], uref[b], kind)
                worst[3] = max(worst[3], (np.linalg.norm(g[b] - gfd) - 1e-8) / np.linalg.norm(gfd))
        print(f"kind {kind}: rho {worst[0]:.1e}, f {worst[1]:.1e}, grad vs torch {worst[2]:.1e}, "
              f"vs FD {worst[3]:.1e}", flush=True)
        assert worst[0] < 1e-12 and worst[1] < 1e-12 and worst[2] < 1e-10 and worst[3] < 1e-6
        del rho, k4
    # the Wootters mixing is a stationary point with f = C^2 / 2
    uo, cc = [], []
    for i in range(len(sample)):
        r = CO.rho_from_theta(ths[i])
        om = OU.optimal_mixing(r / np.trace(r).real, k)
        uo.append(om["W"].T)
        cc.append(om["C"])
    uo = torch.as_tensor(np.stack(uo)).cuda()
    p0 = torch.zeros((len(sample), 16), dtype=torch.float64, device="cuda")
    tsub = th[sidx].contiguous()
    f, rho, k4 = M.unravel_cost(tsub, k, p0, uo, 0)
    g = M.unravel_cost_grad(rho, k4, p0, uo, 0, None)
    cc = np.asarray(cc)
    assert np.abs(f.cpu().numpy() - cc * cc / 2).max() < 1e-12
    assert g.abs().max().item() < 1e-8
    del th
    torch.cuda.empty_cache()
