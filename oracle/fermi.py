"""Fermi-Dirac occupations and their first-order perturbation factors.

Test infrastructure (see the package docstring).

Sec. II.C gives the ground-state density matrix in the orthogonalized basis
as the Fermi-Dirac function of H-perp, D-perp = [exp(beta (H-perp - mu I)) + I]^-1,
with the chemical potential mu fixed by the total electron count summed over
both spin channels. The printed formula drops beta = 1/kT; we restore it.
One mu is shared by both spins (the particle-number constraint is a single
sum over sigma in Sec. II.C and in the constrained minimizations of Sec. III.A).
"""

from __future__ import annotations

import numpy as np


def fermi(eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """f(eps) = 1 / (1 + exp((eps - mu)/kT))."""
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp((np.asarray(eps) - mu) / kT))


def fermi_complement(eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """1 - f(eps), evaluated as f with the sign of (eps - mu) flipped (no cancellation)."""
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-(np.asarray(eps) - mu) / kT))


def electron_count(eps_list, mu: float, kT: float) -> float:
    """Sum over spin channels and levels of f(eps)."""
    return float(sum(fermi(e, mu, kT).sum() for e in eps_list))


def solve_mu(eps_list, n_electrons: float, kT: float, tol: float = 1e-13) -> float:
    """Chemical potential with sum_sigma sum_k f(eps_k^sigma) = N_e.

    Bisection on [min eps - 40 kT, max eps + 40 kT] (the count is monotone in
    mu), then Newton steps with dN/dmu = sum beta f (1 - f).
    """
    lo = min(float(np.min(e)) for e in eps_list) - 40.0 * kT
    hi = max(float(np.max(e)) for e in eps_list) + 40.0 * kT
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if electron_count(eps_list, mid, kT) < n_electrons:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15 * max(1.0, abs(mid)):
            break
    mu = 0.5 * (lo + hi)
    for _ in range(3):
        resid = electron_count(eps_list, mu, kT) - n_electrons
        slope = sum((fermi(e, mu, kT) * fermi_complement(e, mu, kT)).sum() for e in eps_list) / kT
        if slope <= 0.0 or abs(resid) <= tol * n_electrons:
            break
        mu -= resid / slope
    return mu


def phi(z: np.ndarray) -> np.ndarray:
    """phi(z) = (exp(z) - 1)/z, with phi(0) = 1."""
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0.0
    out[nz] = np.expm1(z[nz]) / z[nz]
    return out


def divided_difference_matrix(eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """F_ij = (f_i - f_j)/(eps_i - eps_j), F_ii = f'(eps_i) = -beta f_i (1 - f_i).

    First-order change of the Fermi function of a symmetric matrix in its
    eigenbasis (Daleckii-Krein): d f(H)_ij = F_ij dH_ij. Written without
    cancellation: with a = beta(eps_lo - mu), b = beta(eps_hi - mu), a <= b,
    f(a) - f(b) = f(a) (1 - f(b)) (1 - exp(a - b)), so
    F = -beta f(a) (1 - f(b)) phi(a - b), finite for every gap including ties.
    """
    beta = 1.0 / kT
    e = np.asarray(eps, dtype=np.float64)
    lo = np.minimum(e[:, None], e[None, :])
    hi = np.maximum(e[:, None], e[None, :])
    return -beta * fermi(lo, mu, kT) * fermi_complement(hi, mu, kT) * phi(beta * (lo - hi))
