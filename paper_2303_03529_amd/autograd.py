"""torch.autograd interface of the differentiation form of the Krylov kernel.

KrylovKernel is a torch.autograd.Function whose backward is the hand-written
reverse pass of the HIP library (krylov_kernel_adjoint): gradients of any
scalar L(K delta) with respect to delta, gamma, W and the two expansion-point
spin Hamiltonians H^sigma (Sec. II.G for the kernel, Sec. II.C for how the
expansion point enters). The per-direction response matrices are recomputed
in the reverse sweep, not stored.

kernel_from_parameters builds gamma(U) and H^sigma(H0, gamma, W, n) with
ordinary torch operations on the device (the caller side of the library
boundary, as in caller_setup) and applies KrylovKernel, so torch.autograd
returns dL/dU, dL/dW and dL/dH0 as well:

  gamma_IJ = h / sqrt(r_IJ^2 + (h/U)^2), gamma_II = U   (h = 1 Hartree in eV,
             r in Bohr; the screened Coulomb form of the synthetic Fe model)
  u^sigma  = gamma n_q + s_sigma W n_m,  H^sigma = H0 + 1/2 (U~ S + S U~)   (Sec. III.A)

Energies are in eV. The forward's eigensolve of Z^T H^sigma Z (Z = S^-1/2)
is caller-side setup too (torch.linalg.eigh), as for kk_prepare in general.
With precision KK_MIXED_F16 the forward expansion runs on the split FP16
transforms; the reverse sweep runs split as well when no gradient with respect
to the spin Hamiltonians (hence U, W through them, H0) is needed, and in FP64
otherwise.
"""

from __future__ import annotations

import numpy as np
import torch

from . import krylov


class KernelSystem:
    """Fixed data of one system (S, Z, offsets, distances, n) and its library handle."""

    def __init__(self, sysd: dict, n=None, device: str = "cuda", precision: int = krylov.KK_FP64):
        dt = torch.float64
        self.device = device
        self.precision = precision
        self.offsets = np.asarray(sysd["offsets"], dtype=np.int32)
        self.N = len(self.offsets) - 1
        self.counts = torch.as_tensor(np.diff(self.offsets).astype(np.int64), device=device)
        self.S = torch.as_tensor(sysd["S"], dtype=dt, device=device).contiguous()
        lam, U = torch.linalg.eigh(self.S)
        self.Z = ((U * lam.rsqrt()) @ U.T).contiguous()
        self.r2 = torch.as_tensor(sysd["r2_bohr"], dtype=dt, device=device)
        self.hartree_ev = float(sysd["hartree_ev"])
        self.kT = float(sysd["kT"])
        self.n_electrons = float(sysd["n_electrons"])
        self.n = torch.as_tensor(sysd["n_ref"] if n is None else n, dtype=dt, device=device)
        self.handle = krylov.Handle()
        self.token = 0  # changes with every prepare or kernel call on the handle

    def close(self):
        self.handle.close()

    def gamma_of_U(self, U):
        g = self.hartree_ev / torch.sqrt(self.r2 + (self.hartree_ev / U) ** 2)
        eye = torch.eye(self.N, dtype=torch.bool, device=self.device)
        return torch.where(eye, U * torch.ones_like(g), g)

    def spin_hamiltonians(self, H0, gamma, W):
        Hs = 0.5 * (H0 + H0.T)
        out = []
        for s in (1.0, -1.0):
            u = gamma @ self.n[: self.N] + s * W * self.n[self.N:]
            ut = torch.repeat_interleave(u, self.counts)
            out.append(Hs + 0.5 * (ut[:, None] * self.S + self.S * ut[None, :]))
        return out

    def prepare(self, gamma, W: float, H_up, H_dn):
        """Eigensolve Z^T H^sigma Z and kk_prepare the handle; returns the eigenpairs."""
        eig = []
        for H in (H_up, H_dn):
            Hp = self.Z.T @ H @ self.Z
            e, Q = torch.linalg.eigh(0.5 * (Hp + Hp.T))
            eig += [e.contiguous(), Q.contiguous()]
        e_up, Q_up, e_dn, Q_dn = eig
        self.handle.prepare(self.offsets, self.S, self.Z, Q_up, Q_dn, e_up, e_dn, gamma.contiguous(), W,
                            self.kT, self.n_electrons, self.precision)
        self.token += 1
        return eig


class KrylovKernel(torch.autograd.Function):
    """x = K delta at the expansion point H^sigma; backward through krylov_kernel_adjoint."""

    @staticmethod
    def forward(ctx, delta, gamma, W, H_up, H_dn, system: KernelSystem, m: int):
        with torch.no_grad():
            gamma_c = gamma.detach().contiguous()
            eig = system.prepare(gamma_c, float(W), H_up.detach(), H_dn.detach())
            x, _ = system.handle.krylov_kernel_apply(delta.detach().contiguous(), m, info=False)
            system.token += 1
        ctx.system, ctx.m, ctx.token, ctx.W = system, m, system.token, float(W)
        ctx.save_for_backward(delta.detach().contiguous(), gamma_c, *eig)
        return x.clone()

    @staticmethod
    def backward(ctx, x_bar):
        system = ctx.system
        delta, gamma, e_up, Q_up, e_dn, Q_dn = ctx.saved_tensors
        reuse = system.token == ctx.token
        if not reuse:  # the handle moved on: prepare this expansion point again
            system.handle.prepare(system.offsets, system.S, system.Z, Q_up, Q_dn, e_up, e_dn, gamma, ctx.W,
                                  system.kT, system.n_electrons, system.precision)
        want_H = ctx.needs_input_grad[3] or ctx.needs_input_grad[4]
        g = system.handle.krylov_kernel_adjoint(delta, ctx.m, x_bar.contiguous(), reuse_forward=reuse,
                                                want_H=want_H)
        system.token += 1
        return g["delta"], g["gamma"], g["W"], g["H_up"], g["H_dn"], None, None


def kernel_from_parameters(system: KernelSystem, delta, U, W, H0, m: int):
    """K delta as a differentiable function of delta, U (eV), W (eV) and H0 (tensors)."""
    gamma = system.gamma_of_U(U)
    H_up, H_dn = system.spin_hamiltonians(H0, gamma, W)
    return KrylovKernel.apply(delta, gamma, W, H_up, H_dn, system, m)
