"""GPU cost across the block's internal bond and its hand-written adjoint against the oracle
(cost from the branch tensors' Gram matrices, torch-CPU autograd gradient, central finite
differences) on block shapes that fill one 32-row Gram tile, several tiles, and ragged tiles;
the two-qubit block against the noisy-qubit cost; the autograd wrapper."""
import numpy as np
import pytest

from oracle import cost as CO
from paper_2508_05745_amd import inputs as I

pytestmark = pytest.mark.gpu


def _inputs(B, cl, cr, dtype, seed):
    npdt = np.complex64 if dtype == "c64" else np.complex128
    th = I.random_two_site_states(B, cl, cr, seed=seed, dtype=npdt)
    params = I.random_mixing_params(B, seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    uref = np.stack([I.haar_unitary(rng, 4) for _ in range(B)])
    return th, params, uref


def _moments_ref(th):
    """Normalised rho_q and the 4 x 4 moment matrix of the block Gram, written out."""
    t = th.astype(np.complex128)
    t = t / np.linalg.norm(t)
    cl = t.shape[0]
    x = t.reshape(cl, 2, -1)
    g = np.einsum("ask,bwk->asbw", x, x.conj())                  # Gamma[(a,s),(b,w)]
    rho = np.einsum("asaw->sw", g)
    n = np.einsum("awbx,aybz->wxyz", g, g.conj()).reshape(4, 4)
    return rho, n


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("cl,cr", [(3, 5), (16, 16), (24, 40), (40, 24), (64, 64)])
def test_bond_cost_and_gradient_vs_oracle(kind, dtype, cl, cr):
    import torch

    from paper_2508_05745_amd import mpsb as M
    B = 12
    th, params, uref = _inputs(B, cl, cr, dtype, 5000 + cl + 7 * cr)
    k = I.amplitude_damping(0.3) if kind else I.depolarizing(0.1)
    pp = torch.as_tensor(params).cuda()
    uu = torch.as_tensor(uref).cuda()
    f, rho, nm, k4 = M.unravel_cost_bond(torch.as_tensor(th).cuda(), k, pp, uu, kind)
    g = M.unravel_cost_bond_grad(rho, nm, k4, pp, uu, kind, None)
    f, rho, nm, g = (x.cpu().numpy() for x in (f, rho, nm, g))
    print(f"bond cost {dtype} {cl}x{cr} kind {kind}", flush=True)
    for b in range(B):
        r_ref, n_ref = _moments_ref(th[b])
        assert np.abs(rho[b] - r_ref).max() < 1e-13
        assert np.abs(nm[b] - n_ref).max() < 1e-13
        f_ref, g_ref = CO.bond_grad_torch(th[b], k, params[b], uref[b], kind)
        assert abs(f[b] - f_ref) < 1e-12, (b, f[b], f_ref)
        assert np.linalg.norm(g[b] - g_ref) <= 1e-10 * max(1.0, np.linalg.norm(g_ref))
    gfd = CO.bond_grad_fd(th[0], k, params[0], uref[0], kind)
    assert np.linalg.norm(g[0] - gfd) <= 1e-6 * np.linalg.norm(gfd) + 1e-8


@pytest.mark.parametrize("kind", [0, 1])
def test_two_qubit_block_equals_noisy_qubit_cost(kind):
    import torch

    from paper_2508_05745_amd import mpsb as M
    B = 256
    th, params, uref = _inputs(B, 1, 1, "c128", 77)
    k = I.depolarizing(0.3)
    tt, pp, uu = (torch.as_tensor(x).cuda() for x in (th, params, uref))
    fb, rb, nb, k4 = M.unravel_cost_bond(tt, k, pp, uu, kind)
    gb = M.unravel_cost_bond_grad(rb, nb, k4, pp, uu, kind, None)
    fa, ra, k4a = M.unravel_cost(tt, k, pp, uu, kind)
    ga = M.unravel_cost_grad(ra, k4a, pp, uu, kind, None)
    assert (fb - fa).abs().max().item() < 1e-13
    assert (gb - ga).abs().max().item() < 1e-12


def test_bond_autograd_function_and_edges():
    import torch

    from paper_2508_05745_amd import mpsb as M
    B = 8
    th, params, uref = _inputs(B, 8, 12, "c128", 91)
    k = I.dephasing(0.2)
    pp = torch.as_tensor(params).cuda().requires_grad_(True)
    UC = M.UnravelCost(bond=True)
    w = torch.linspace(0.5, 2.0, B, dtype=torch.float64, device="cuda")
    f = UC.apply(pp, torch.as_tensor(th).cuda(), k, torch.as_tensor(uref).cuda(), 1)
    (w * f).sum().backward()
    g = pp.grad.cpu().numpy()
    wc = w.cpu().numpy()
    for b in range(B):
        _, g_ref = CO.bond_grad_torch(th[b], k, params[b], uref[b], 1)
        assert np.linalg.norm(g[b] - wc[b] * g_ref) <= 1e-10 * max(1.0, np.linalg.norm(g_ref))
    # an empty batch is a no-op; bad sizes and kinds are refused
    e = torch.zeros((0, 4, 2, 2, 4), dtype=torch.complex128, device="cuda")
    out = M.unravel_cost_bond(e, k, torch.zeros((0, 16), dtype=torch.float64, device="cuda"),
                              torch.zeros((0, 4, 4), dtype=torch.complex128, device="cuda"), 0)
    assert out[0].numel() == 0
    with pytest.raises(M.MpsbError):
        M.unravel_cost_bond(torch.as_tensor(th).cuda(), k, pp.detach(), torch.as_tensor(uref).cuda(), 2)


def test_bond_cost_at_full_size_sampled():
    """The benchmark's workload and launch shape (16384 chi-64 c64 states drawn on the device,
    one wave per state): sampled states against the oracle, and every cost finite and within
    the bounds of a linear entropy across a cut of dimension 2 chi: 0 <= f <= 1 - 1 / (2 chi)."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    B, chi = 16384, 64
    th = I.random_two_site_states_torch(B, chi, chi, seed=4004)
    pp = torch.as_tensor(I.random_mixing_params(B, seed=4005)).cuda()
    uu = torch.as_tensor(I.haar_unitaries(B, seed=4006)).cuda()
    k = I.depolarizing(0.02)
    f, rho, nm, k4 = M.unravel_cost_bond(th, k, pp, uu, 0)
    g = M.unravel_cost_bond_grad(rho, nm, k4, pp, uu, 0, None)
    fc = f.cpu().numpy()
    assert np.isfinite(fc).all() and fc.min() >= 0.0 and fc.max() <= 1.0 - 1.0 / (2 * chi)
    sample = [0, 1, 4095, 8191, 12000, B - 1]
    ths = th[torch.as_tensor(sample).cuda()].cpu().numpy()
    gc, params, uref = g.cpu().numpy(), pp.cpu().numpy(), uu.cpu().numpy()
    for i, b in enumerate(sample):
        f_ref, g_ref = CO.bond_grad_torch(ths[i], k, params[b], uref[b], 0)
        assert abs(fc[b] - f_ref) < 1e-12
        assert np.linalg.norm(gc[b] - g_ref) <= 1e-10 * max(1.0, np.linalg.norm(g_ref))
