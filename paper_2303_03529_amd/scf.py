"""Kernel-accelerated SCF and extended-Lagrangian electronic steps on the GPU.

Sec. III.C: the quasi-Newton SCF n_new = n_old - K (q[n_old] - n_old) with K
the preconditioned low-rank Krylov kernel at the current n (a few ranks per
step, chosen adaptively), against a plain linear mixer n_new = n_old +
a (q[n_old] - n_old); the kernel mixer starts once the charge error is below
`switch_at`. Sec. II.F: n(t+dt) = 2 n - n(t-dt) - kappa K f + alpha sum c_k n(t-k dt).

Every step runs in the HIP library: the ground-state map q[n]
(kk_ground_state_charges after kk_prepare), the kernel
(krylov_kernel_apply_adaptive) and the n updates (kk_xlbomd_update: the
extended-Lagrangian step, and the SCF mixer steps as that update with
n(t - dt) = n(t), alpha = 0, so 2 n - n - kappa v = n - kappa v: kappa = 1,
v = K f for the kernel mixer; kappa = -a, v = f for the linear one). The
caller side (DeviceSystem) builds and diagonalizes the spin Hamiltonians.
Charges are net Mulliken charges (neutral-atom valence subtracted,
Sec. III.A); the host only keeps the loop, the residual q[n] - n and the
convergence test.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import krylov
from .caller_setup import DeviceSystem


def net_charges(handle, valence_t) -> torch.Tensor:
    """q[n] - (valence, 0) at the handle's prepared expansion point."""
    return handle.ground_state_charges(valence_t)


def mixer_step(handle, n, v, kappa: float, zero1) -> torch.Tensor:
    """n - kappa v through kk_xlbomd_update with a one-row history (n(t - dt) = n(t), alpha = 0)."""
    return handle.xlbomd_update(n[None, :].contiguous(), v.contiguous(), kappa, 0.0, zero1)


def scf(sysd: dict, n0, mixer: str = "kernel", tol: float = 1e-8, max_iter: int = 100, m_max: int = 8,
        rank_tol: float = 0.1, linear_coeff: float = 0.06, switch_at: float = 0.05,
        precision: int = krylov.KK_FP64, device: str = "cuda"):
    """Returns (n as numpy, history of dicts with rms residual, rank, mode)."""
    ds = DeviceSystem(sysd, device)
    h = krylov.Handle()
    valence = torch.as_tensor(sysd["valence"], dtype=torch.float64, device=device)
    n = torch.as_tensor(np.asarray(n0, dtype=np.float64), device=device).clone()
    zero1 = torch.zeros(1, dtype=torch.float64, device=device)
    hist = []
    try:
        for _ in range(max_iter):
            ds.prepare(h, n, precision)
            f = net_charges(h, valence) - n
            err = float(torch.sqrt(torch.mean(f * f)))
            if err <= tol:
                hist.append(dict(rms=err, rank=0, mode="done"))
                break
            if mixer == "linear" or err > switch_at:
                hist.append(dict(rms=err, rank=0, mode="linear"))
                n = mixer_step(h, n, f, -linear_coeff, zero1)
                continue
            Kf, info = h.krylov_kernel_apply_adaptive(f.contiguous(), m_max, rank_tol)
            hist.append(dict(rms=err, rank=info.rank_used, mode="kernel", ls_residual=info.ls_residual))
            n = mixer_step(h, n, Kf, 1.0, zero1)
    finally:
        h.close()
    return n.cpu().numpy(), hist


def xlbomd_electrons(sysd: dict, n_start, steps: int, kappa: float, alpha: float = 0.0, c=(1.0,),
                     m_max: int = 4, rank_tol: float = 0.1, precision: int = krylov.KK_FP64,
                     device: str = "cuda", return_residuals: bool = False):
    """Propagate n with the extended-Lagrangian update at fixed nuclei.

    n(t) and its history start at n_start. Each step prepares q[n(t)], applies
    the adaptive-rank kernel to f = q[n] - n and calls kk_xlbomd_update.
    Returns the rms residual per step and the final n (and, with
    return_residuals, the residual vectors per step).
    """
    ds = DeviceSystem(sysd, device)
    h = krylov.Handle()
    valence = torch.as_tensor(sysd["valence"], dtype=torch.float64, device=device)
    kmax = max(len(c) - 1, 1)
    n0 = torch.as_tensor(np.asarray(n_start, dtype=np.float64), device=device)
    hist = n0.repeat(kmax + 1, 1).contiguous()           # rows n(t - k dt)
    cc = torch.zeros(kmax + 1, dtype=torch.float64, device=device)
    cc[: len(c)] = torch.as_tensor(c, dtype=torch.float64)
    out, fs = [], []
    try:
        for _ in range(steps):
            n = hist[0].contiguous()
            ds.prepare(h, n, precision)
            f = (net_charges(h, valence) - n).contiguous()
            out.append(float(torch.sqrt(torch.mean(f * f))))
            fs.append(f.cpu().numpy())
            Kf, _ = h.krylov_kernel_apply_adaptive(f, m_max, rank_tol)
            n_new = h.xlbomd_update(hist, Kf, kappa, alpha, cc)
            hist = torch.cat([n_new[None, :], hist[:-1]], dim=0).contiguous()
    finally:
        h.close()
    if return_residuals:
        return out, hist[0].cpu().numpy(), fs
    return out, hist[0].cpu().numpy()


def rms(x) -> float:
    return math.sqrt(float(np.mean(np.asarray(x) ** 2)))
