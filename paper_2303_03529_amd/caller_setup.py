"""Caller-side expansion point on the device (outside the library boundary).

An MD or SCF driver diagonalizes its spin Hamiltonians once per step and hands
(Z, Q, eps) to kk_prepare; the library starts from there. This helper does
that step for synthetic systems with torch.linalg on the GPU:
  H^sigma = H0 + 1/2 (U~ S + S U~), u^sigma = gamma n_q + s_sigma W n_m  (Sec. III.A)
  Z = S^-1/2 (Loewdin), eigenpairs of Z^T H^sigma Z                      (Sec. II.C)
"""

from __future__ import annotations

import numpy as np
import torch


def expansion_point_device(sysd: dict, device="cuda", n=None) -> dict:
    dt = torch.float64
    N = sysd["gamma"].shape[0]
    n = sysd["n_ref"] if n is None else n
    counts = np.diff(sysd["offsets"])
    S = torch.as_tensor(sysd["S"], dtype=dt, device=device)
    H0 = torch.as_tensor(sysd["H0"], dtype=dt, device=device)
    gamma = torch.as_tensor(sysd["gamma"], dtype=dt, device=device)
    lam, U = torch.linalg.eigh(S)
    Z = (U * lam.rsqrt()) @ U.T
    out = dict(S=S, Z=Z.contiguous(), gamma=gamma.contiguous())
    for name, sgn in (("up", 1.0), ("dn", -1.0)):
        u = gamma @ torch.as_tensor(n[:N], dtype=dt, device=device) \
            + sgn * sysd["W"] * torch.as_tensor(n[N:], dtype=dt, device=device)
        ut = torch.repeat_interleave(u, torch.as_tensor(counts, device=device))
        H = H0 + 0.5 * (ut[:, None] * S + S * ut[None, :])
        Hp = Z.T @ H @ Z
        Hp = 0.5 * (Hp + Hp.T)
        e, Q = torch.linalg.eigh(Hp)
        out["eps_" + name] = e.contiguous()
        out["Q_" + name] = Q.contiguous()
    return out
