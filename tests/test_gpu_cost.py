"""GPU unravelling cost and its hand-written adjoint against the oracle (float64 cost from
the oracle's own reduced state, torch-CPU autograd gradient, central finite differences),
the optimum (f = C^2/2, zero gradient), and the torch.autograd.Function wrapper."""
import numpy as np
import pytest

from oracle import cost as CO
from oracle import unravel as OU
from paper_2508_05745_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_cost_and_gradient_vs_oracle(kind, dtype):
    import torch

    from paper_2508_05745_amd import mpsb as M
    B = 64
    npdt = np.complex64 if dtype == "c64" else np.complex128
    th = I.random_two_site_states(B, 16, 16, seed=4004, dtype=npdt)
    params = I.random_mixing_params(B, seed=4005)
    rng = np.random.default_rng(4006)
    uref = np.stack([I.haar_unitary(rng, 4) for _ in range(B)])
    k = I.depolarizing(0.02)
    tt = torch.as_tensor(th).cuda()
    pp = torch.as_tensor(params).cuda()
    uu = torch.as_tensor(uref).cuda()
    f, rho, k4 = M.unravel_cost(tt, k, pp, uu, kind)
    g = M.unravel_cost_grad(rho, k4, pp, uu, kind, None)
    f, rho, g = f.cpu().numpy(), rho.cpu().numpy(), g.cpu().numpy()
    for b in range(B):
        r_ref = CO.rho_from_theta(th[b])
        assert np.abs(rho[b] - r_ref).max() < 1e-12
        f_ref, g_ref = CO.grad_torch(r_ref / np.trace(r_ref).real, k, params[b], uref[b], kind)
        assert abs(f[b] - f_ref) < 1e-12
        assert np.linalg.norm(g[b] - g_ref) <= 1e-10 * max(1.0, np.linalg.norm(g_ref))
    for b in range(4):
        r_ref = CO.rho_from_theta(th[b])
        gfd = CO.grad_fd(r_ref / np.trace(r_ref).real, k, params[b], uref[b], kind)
        assert np.linalg.norm(g[b] - gfd) <= 1e-6 * np.linalg.norm(gfd) + 1e-8


def test_optimum_and_autograd_function():
    import torch

    from paper_2508_05745_amd import mpsb as M
    B = 32
    th = I.random_two_site_states(B, 8, 8, seed=17, dtype=np.complex128)
    k = I.depolarizing(0.02)
    uo = []
    for b in range(B):
        r = CO.rho_from_theta(th[b])
        uo.append(OU.optimal_mixing(r / np.trace(r).real, k)["W"].T)
    uo = torch.as_tensor(np.stack(uo)).cuda()
    params = torch.zeros((B, 16), dtype=torch.float64, device="cuda", requires_grad=True)
    tt = torch.as_tensor(th).cuda()
    UC = M.UnravelCost()
    f = UC.apply(params, tt, k, uo, 0)
    f.sum().backward()
    fc = f.detach().cpu().numpy()
    for b in range(B):
        r = CO.rho_from_theta(th[b])
        c = OU.optimal_mixing(r / np.trace(r).real, k)["C"]
        assert abs(fc[b] - c * c / 2) < 1e-12
    assert params.grad.abs().max().item() < 1e-8
