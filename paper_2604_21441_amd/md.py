"""NVE velocity-Verlet driver on top of the library (microcanonical MD with the
NNP as the only force field; the paper's water-box benchmark runs NVE, see its
performance section).

Master positions and velocities are FP64 on the device; each step casts the
positions to FP32 for ``nnp_compute`` (which reruns the neighbour search) and
records E_pot and the kinetic energy on the device; everything is read back
once at the end.  Units: A, fs, amu, eV.
"""
from __future__ import annotations

import time

import numpy as np
import torch

ACC_UNIT = 9.64853321233e-3   # 1 eV / (A amu) in A / fs^2


def run_nve(model, pos, Z, box, masses, v0, dt: float = 0.5, steps: int = 1000, stream=None):
    """Integrate `steps` velocity-Verlet steps of length dt (fs).

    model : NNPModel; pos [n, 3] (A), v0 [n, 3] (A/fs), masses [n] (amu).
    Returns dict(t [steps+1] fs, epot, ekin, etot [eV], drift_eV_per_atom_per_ps (slope of a
    least-squares line through etot / n), max_abs_dev_eV_per_atom, ms_per_step).
    """
    dev = torch.device("cuda")
    n = pos.shape[0]
    x = torch.as_tensor(np.asarray(pos, np.float64), device=dev).clone()
    v = torch.as_tensor(np.asarray(v0, np.float64), device=dev).clone()
    m = torch.as_tensor(np.asarray(masses, np.float64), device=dev)[:, None]
    x32 = x.float()
    E = torch.empty(1, dtype=torch.float64, device=dev)
    F = torch.empty((n, 3), dtype=torch.float64, device=dev)
    epot = torch.empty(steps + 1, dtype=torch.float64, device=dev)
    ekin = torch.empty(steps + 1, dtype=torch.float64, device=dev)

    def kinetic():
        return 0.5 * torch.sum(m * v * v) / ACC_UNIT

    model.compute(x32, Z, box, out=(E, F, None), stream=stream)
    a = F / m * ACC_UNIT
    epot[0] = E[0]
    ekin[0] = kinetic()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(1, steps + 1):
        v.add_(a, alpha=0.5 * dt)
        x.add_(v, alpha=dt)
        x32.copy_(x)
        model.compute(x32, None, box, out=(E, F, None), stream=stream)
        torch.div(F, m, out=a)
        a.mul_(ACC_UNIT)
        v.add_(a, alpha=0.5 * dt)
        epot[s] = E[0]
        ekin[s] = kinetic()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if model.status() != 0:
        raise RuntimeError("the NNP reported a device-side error during the run")
    ep = epot.cpu().numpy()
    ek = ekin.cpu().numpy()
    et = ep + ek
    t = np.arange(steps + 1) * dt
    slope = np.polyfit(t, et / n, 1)[0] if steps > 1 else 0.0   # eV/atom/fs
    return {"t": t, "epot": ep, "ekin": ek, "etot": et,
            "drift_eV_per_atom_per_ps": float(slope * 1000.0),
            "max_abs_dev_eV_per_atom": float(np.max(np.abs(et - et[0])) / n),
            "ms_per_step": wall * 1e3 / max(steps, 1)}
