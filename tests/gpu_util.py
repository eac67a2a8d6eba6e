"""Helpers shared by the GPU parity tests (running the HIP path and the oracle on the same
seeded inputs)."""
import numpy as np

from oracle import mps as omps
from oracle import sv as osv


def run_gpu(circuit, chi, n_traj, seed, precision, mode, fixed_u=None, record=False):
    import torch

    from paper_2508_05745_amd import mpsb as M
    b = M.Batch(n_traj, circuit.n, chi, precision, seed)
    b.set_circuit(circuit, mode, fixed_u)
    ws, brs, disc = [], [], []
    w = torch.zeros((n_traj, circuit.n, 4, 4), dtype=torch.complex128, device="cuda") if record else None
    br = torch.zeros((n_traj, circuit.n), dtype=torch.int32, device="cuda") if record else None
    d = torch.zeros((n_traj, circuit.n // 2), dtype=torch.float64, device="cuda") if record else None
    for l in range(circuit.depth):
        b.apply_layer(l, discarded=d, branch=br, w_record=w)
        if record:
            ws.append(w.cpu().numpy().copy())
            brs.append(br.cpu().numpy().copy())
            disc.append(d.cpu().numpy().copy())
    mean, m2, pt = b.expect()
    b.sync()
    out = dict(mean=mean.cpu().numpy(), m2=m2.cpu().numpy(), per_traj=pt.cpu().numpy(),
               w=ws, branch=brs, disc=disc)
    b.close()
    return out


def recorded_events(circuit, out, t):
    """GPU-recorded W (as r x 4 'W' matrices) and branches of trajectory t, in the oracle's
    event order."""
    ws, js = [], []
    for l in range(circuit.depth):
        for kind, q in osv.sweep_ops(circuit, l):
            for x in osv.event_qubits(circuit, l, kind, q):
                ws.append(out["w"][l][t, x].T.copy())
                js.append(int(out["branch"][l][t, x]))
    return ws, js


def oracle_obs_sv(circuit, t, seed, mode, fixed_u=None, replay=None, record=None):
    psi = osv.trajectory(circuit, t, seed, mode=mode, fixed_u=fixed_u, replay=replay, record=record)
    zi, zz = osv.z_expectations(psi, circuit.n)
    return np.concatenate([zi, zz])


def oracle_obs_mps(circuit, chi, t, seed, mode, fixed_u=None, replay=None, record=None):
    m, eps = omps.trajectory(circuit, chi, t, seed, mode=mode, fixed_u=fixed_u, replay=replay,
                             record=record)
    zi, zz = omps.z_expectations(m)
    return np.concatenate([zi, zz]), eps


def run_gpu_sampled(circuit, chi, n_traj, seed, precision, mode, layers, sample):
    """Run `layers` brickwork layers on the whole batch (the launch configuration of a
    production run) and keep the recorded mixings / branches / observables of the sampled
    trajectories only."""
    import torch

    from paper_2508_05745_amd import mpsb as M
    b = M.Batch(n_traj, circuit.n, chi, precision, seed)
    b.set_circuit(circuit, mode)
    idx = torch.as_tensor(list(sample), device="cuda")
    w = torch.zeros((n_traj, circuit.n, 4, 4), dtype=torch.complex128, device="cuda")
    br = torch.zeros((n_traj, circuit.n), dtype=torch.int32, device="cuda")
    ws, brs = [], []
    for l in range(layers):
        b.apply_layer(l, branch=br, w_record=w)
        ws.append(w[idx].cpu().numpy())
        brs.append(br[idx].cpu().numpy())
    mean, m2, pt = b.expect()
    b.sync()
    out = dict(mean=mean.cpu().numpy(), m2=m2.cpu().numpy(), per_traj=pt[idx].cpu().numpy(),
               all_per_traj=pt.cpu().numpy(), w=ws, branch=brs, sample=list(sample), layers=layers)
    b.close()
    del w, br, pt, mean, m2
    torch.cuda.empty_cache()
    return out


def replay_sampled(circuit, chi, seed, out, row):
    """Oracle MPS replay of sampled trajectory out['sample'][row] over out['layers'] layers:
    returns (oracle observables, Replay object, GPU branches, oracle branches, singular-value
    spectra of every split)."""
    t = out["sample"][row]
    ws, js = [], []
    for l in range(out["layers"]):
        for kind, q in osv.sweep_ops(circuit, l):
            for x in osv.event_qubits(circuit, l, kind, q):
                ws.append(out["w"][l][row, x].T.copy())
                js.append(int(out["branch"][l][row, x]))
    rp = osv.Replay(ws)
    rec, spectra = [], []
    m, _ = omps.trajectory(circuit, chi, t, seed, mode=3, layers=out["layers"], record=rec, replay=rp,
                           spectra=spectra)
    zi, zz = omps.z_expectations(m)
    return np.concatenate([zi, zz]), rp, js, [r["j"] for r in rec], spectra
