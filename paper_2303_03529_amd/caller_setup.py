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


class DeviceSystem:
    """Device copies of one system's H0, S, gamma and its Loewdin factor Z."""

    def __init__(self, sysd: dict, device="cuda"):
        dt = torch.float64
        self.sysd = sysd
        self.device = device
        self.N = sysd["gamma"].shape[0]
        self.S = torch.as_tensor(sysd["S"], dtype=dt, device=device)
        self.H0 = torch.as_tensor(sysd["H0"], dtype=dt, device=device)
        self.gamma = torch.as_tensor(sysd["gamma"], dtype=dt, device=device).contiguous()
        self.counts = torch.as_tensor(np.diff(sysd["offsets"]), device=device)
        lam, U = torch.linalg.eigh(self.S)
        self.Z = ((U * lam.rsqrt()) @ U.T).contiguous()

    def expansion(self, n=None) -> dict:
        """Z, Q_s, eps_s of the spin Hamiltonians at n (default: the system's n_ref)."""
        dt = torch.float64
        n = self.sysd["n_ref"] if n is None else n
        n = torch.as_tensor(n, dtype=dt, device=self.device)
        out = dict(S=self.S, Z=self.Z, gamma=self.gamma)
        for name, sgn in (("up", 1.0), ("dn", -1.0)):
            u = self.gamma @ n[: self.N] + sgn * self.sysd["W"] * n[self.N:]
            ut = torch.repeat_interleave(u, self.counts)
            H = self.H0 + 0.5 * (ut[:, None] * self.S + self.S * ut[None, :])
            Hp = self.Z.T @ H @ self.Z
            Hp = 0.5 * (Hp + Hp.T)
            e, Q = torch.linalg.eigh(Hp)
            out["eps_" + name] = e.contiguous()
            out["Q_" + name] = Q.contiguous()
        return out

    def prepare(self, handle, n=None, precision: int = 0):
        """kk_prepare the library handle at n."""
        e = self.expansion(n)
        handle.prepare(self.sysd["offsets"], e["S"], e["Z"], e["Q_up"], e["Q_dn"], e["eps_up"], e["eps_dn"],
                       e["gamma"], self.sysd["W"], self.sysd["kT"], self.sysd["n_electrons"], precision)
        return handle


def expansion_point_device(sysd: dict, device="cuda", n=None) -> dict:
    return DeviceSystem(sysd, device).expansion(n)
