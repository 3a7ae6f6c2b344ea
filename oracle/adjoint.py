"""Gradients of L = ||K delta||^2 with respect to delta, U, W and H0.

Test infrastructure (see the package docstring).

The differentiation form asks for the derivatives of the squared norm of
the rank-m Krylov kernel result, L = ||K delta||^2, with respect to the
residual delta, the Hubbard U (through gamma), the Stoner constant W and the
charge-independent Hamiltonian H0, at a fixed expansion point n (Sec. II.G
for the kernel, Sec. III.A for how U, W and H0 enter).

This module writes L(delta, U, W, H0) out as plain torch float64 CPU
operations in the order of the definitions and lets torch.autograd
differentiate it. It is a generic reverse-mode derivative of the plain
forward (through the eigendecomposition, the chemical-potential condition,
every response and the Gram-Schmidt steps), so it shares nothing with a
hand-derived adjoint. The forward, step by step:

  gamma_IJ(U) = h / sqrt(r_IJ^2 + (h/U)^2), gamma_II = U   (h = 1 Hartree in eV,
                r in Bohr: the screened Coulomb form of the synthetic Fe model)
  u^sigma    = gamma n_q + s_sigma W n_m at the expansion point n
  H^sigma    = H0 + 1/2 (U~ S + S U~)                       (Sec. III.A)
  eps, Q     = eigh(Z^T H^sigma Z), Z = S^-1/2               (Sec. II.C)
  mu         from sum_sigma sum_k f(eps_k) = N_e: solved by bisection, then one
               Newton step taken inside the graph, so that its derivative is
               the implicit-function derivative of the constraint
  q1(v)      the first-order response of oracle.response, restated in torch
  K delta    m Krylov steps with two-pass modified Gram-Schmidt and the
             Cholesky solve of the projected normal equations (oracle.krylov)
  L          = (K delta)^T (K delta)

Gradients with respect to H0 are those of the symmetric matrix: the forward
uses 1/2 (H0 + H0^T), so dL = sum_ij G_ij dH0_ij for every symmetric dH0.
Energies are in eV; U and W are per eV.

Valid away from exactly degenerate levels (the eigh derivative divides by
level gaps) and for a full-rank expansion (rank m reached).
"""

from __future__ import annotations

import numpy as np
import torch

from .expansion import congruence_lowdin
from .fermi import solve_mu

BREAKDOWN_TOL = 1e-13
DT = torch.float64


def gamma_of_U(r2_bohr, U, hartree_ev):
    """Screened Coulomb matrix at Hubbard U (eV) from squared distances in Bohr^2."""
    r2 = torch.as_tensor(r2_bohr, dtype=DT)
    g = hartree_ev / torch.sqrt(r2 + (hartree_ev / U) ** 2)
    eye = torch.eye(r2.shape[0], dtype=torch.bool)
    return torch.where(eye, U * torch.ones_like(g), g)


def _atom_sum(x, offsets):
    """Sum of a per-orbital vector over each atom's orbitals."""
    off = np.asarray(offsets)
    return torch.stack([x[off[a]:off[a + 1]].sum() for a in range(len(off) - 1)])


def _orbital(u, offsets):
    counts = torch.as_tensor(np.diff(np.asarray(offsets)))
    return torch.repeat_interleave(u, counts)


def _fermi_parts(eps, mu, beta):
    """f, 1 - f and the divided-difference matrix F (as in oracle.fermi), in torch."""
    f = torch.sigmoid(-beta * (eps - mu))
    fc = torch.sigmoid(beta * (eps - mu))
    ei, ej = eps[:, None], eps[None, :]
    lo_is_i = ei <= ej
    f_lo = torch.where(lo_is_i, f[:, None], f[None, :])
    fc_hi = torch.where(lo_is_i, fc[None, :], fc[:, None])
    z = beta * -(ei - ej).abs()
    tie = z == 0
    zs = torch.where(tie, -torch.ones_like(z), z)
    phi = torch.where(tie, torch.ones_like(z), torch.expm1(zs) / zs)
    F = -beta * f_lo * fc_hi * phi
    return f, fc, F


def kernel_loss(sysd: dict, delta, U, W, H0, m: int, K0=None, return_parts: bool = False, gamma=None):
    """L = ||K delta||^2 as a torch scalar (all arguments torch tensors on the CPU).

    gamma, if given, is used instead of gamma(U) (to differentiate with respect to
    its entries)."""
    S = torch.as_tensor(sysd["S"], dtype=DT)
    offsets = sysd["offsets"]
    N = sysd["gamma"].shape[0]
    beta = 1.0 / sysd["kT"]
    Z = torch.as_tensor(congruence_lowdin(sysd["S"]), dtype=DT)
    n_ref = torch.as_tensor(sysd["n_ref"], dtype=DT)
    if gamma is None:
        gamma = gamma_of_U(sysd["r2_bohr"], U, sysd["hartree_ev"])
    Hs = 0.5 * (H0 + H0.T)

    # expansion point
    Q, eps = [], []
    for s in (1.0, -1.0):
        u = gamma @ n_ref[:N] + s * W * n_ref[N:]
        ut = _orbital(u, offsets)
        H = Hs + 0.5 * (ut[:, None] * S + S * ut[None, :])
        Hp = Z.T @ H @ Z
        e, q = torch.linalg.eigh(0.5 * (Hp + Hp.T))
        eps.append(e)
        Q.append(q)
    mu0 = solve_mu([e.detach().numpy() for e in eps], sysd["n_electrons"], sysd["kT"])
    count = sum(torch.sigmoid(-beta * (e - mu0)).sum() for e in eps)
    slope = sum((beta * torch.sigmoid(-beta * (e - mu0)) * torch.sigmoid(beta * (e - mu0))).sum() for e in eps)
    mu = mu0 - (count - sysd["n_electrons"]) / slope
    parts = [_fermi_parts(e, mu, beta) for e in eps]
    w = [beta * f * fc for f, fc, _ in parts]
    wsum = w[0].sum() + w[1].sum()

    def response(v):
        X = []
        for s, q in zip((1.0, -1.0), Q):
            u = gamma @ v[:N] + s * W * v[N:]
            ut = _orbital(u, offsets)
            H1 = 0.5 * (ut[:, None] * S + S * ut[None, :])
            X.append(q.T @ (Z.T @ H1 @ Z) @ q)
        dmu = sum((wi * torch.diagonal(Xi)).sum() for wi, Xi in zip(w, X)) / wsum
        dn = []
        for Xi, (_, _, F), wi, q in zip(X, parts, w, Q):
            Y = F * Xi + dmu * torch.diag(wi)
            dD = Z @ q @ Y @ q.T @ Z.T
            dn.append(_atom_sum(torch.diagonal(dD @ S), offsets))
        return torch.cat([dn[0] + dn[1], dn[0] - dn[1]])

    def k0(x):
        return -x if K0 is None else K0 @ x

    ftilde = k0(delta)
    V, Ft = [], []
    r = ftilde
    for _ in range(m):
        wv = r
        start = torch.linalg.norm(wv)
        for _ in range(2):
            for vj in V:
                wv = wv - (vj @ wv) * vj
        nw = torch.linalg.norm(wv)
        if float(nw.detach()) <= BREAKDOWN_TOL * float(start.detach()):
            break
        vk = wv / nw
        ftk = k0(response(vk) - vk)
        V.append(vk)
        Ft.append(ftk)
        r = ftk
    Vm = torch.stack(V, dim=1)
    Fm = torch.stack(Ft, dim=1)
    O = Fm.T @ Fm
    Lc = torch.linalg.cholesky(O)
    c = torch.cholesky_solve((Fm.T @ ftilde)[:, None], Lc)[:, 0]
    x = Vm @ c
    L = x @ x
    if return_parts:
        return L, dict(x=x, rank=len(V), mu=mu)
    return L


def gradients(sysd: dict, m: int, delta=None, U=None, W=None, H0=None, K0=None) -> dict:
    """L and its gradients with respect to delta, U, W and H0 (numpy / float)."""
    d = torch.tensor(sysd["delta"] if delta is None else delta, dtype=DT, requires_grad=True)
    u = torch.tensor(sysd["U"] if U is None else U, dtype=DT, requires_grad=True)
    wv = torch.tensor(sysd["W"] if W is None else W, dtype=DT, requires_grad=True)
    h0 = torch.tensor(sysd["H0"] if H0 is None else H0, dtype=DT, requires_grad=True)
    k0 = None if K0 is None else torch.as_tensor(K0, dtype=DT)
    L, parts = kernel_loss(sysd, d, u, wv, h0, m, k0, return_parts=True)
    gd, gu, gw, gh = torch.autograd.grad(L, [d, u, wv, h0])
    return dict(L=float(L.detach()), delta=gd.numpy(), U=float(gu), W=float(gw), H0=gh.numpy(),
                Kdelta=parts["x"].detach().numpy(), rank=parts["rank"])


def U_gradient_terms(sysd: dict, m: int) -> np.ndarray:
    """The N x N terms dL/dgamma_IJ dgamma_IJ/dU whose sum is dL/dU (chain rule through gamma)."""
    d = torch.tensor(sysd["delta"], dtype=DT)
    u = torch.tensor(sysd["U"], dtype=DT)
    wv = torch.tensor(sysd["W"], dtype=DT)
    h0 = torch.tensor(sysd["H0"], dtype=DT)
    g = gamma_of_U(sysd["r2_bohr"], u, sysd["hartree_ev"]).detach().requires_grad_(True)
    (gg,) = torch.autograd.grad(kernel_loss(sysd, d, u, wv, h0, m, gamma=g), [g])
    h = sysd["hartree_ev"]
    r2 = torch.as_tensor(sysd["r2_bohr"], dtype=DT)
    dg = h * (h * h / u ** 3) / (r2 + (h / u) ** 2) ** 1.5      # d gamma_IJ / dU off the diagonal
    dg = torch.where(torch.eye(r2.shape[0], dtype=torch.bool), torch.ones_like(dg), dg)
    return (gg * dg).detach().numpy()


def U_gradient_scale(sysd: dict, m: int) -> float:
    """sum_IJ |dL/dgamma_IJ dgamma_IJ/dU|: the size of the terms whose sum is dL/dU.

    dL/dU is a strongly cancelling sum (its terms are a few hundred times larger
    than the result on the bcc-Fe systems), so an error bound for it is stated
    relative to this scale."""
    return float(np.abs(U_gradient_terms(sysd, m)).sum())
