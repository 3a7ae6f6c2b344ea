"""Expansion point and the ground-state map n -> q[n].

Test infrastructure (see the package docstring).

Sec. II.C: H-perp = Z^T H Z with Z^T S Z = I (Z = S^-1/2, "or more generally"
any congruence factor), D-perp = Fermi(H-perp), D = Z D-perp Z^T; one
diagonalization, no self-consistency.

Sec. III.A (spin-polarized SCC-DFTB): the linearized shadow energy is
  Tr[H0 (D - D0)] + 1/2 sum_IJ (2 q_I - n_I) gamma_IJ n_J
                   + 1/2 sum_I (2 m_I - s_I) J s_I  - T S,
with Mulliken charge q_I and moment m_I (sums over the atom's orbitals of
(D S)_ii, both spins for q, up minus down for m). Its derivative with
respect to the symmetric D^sigma is the spin Hamiltonian used here:
  H^sigma = H0 + 1/2 (U~ S + S U~),  u^sigma_I = (gamma n_q)_I + s_sigma W (n_m)_I,
with s_up = +1, s_down = -1 and U~ = diag(u^sigma of each orbital's atom).
We take one Stoner constant W for every atom and shell (per-atom moments,
not l-resolved ones), and coordinates n = (n_q, n_m) = (n_up + n_dn, n_up - n_dn).
The constant D0 term of the Mulliken charges drops out of every derivative,
so q[n] below omits it.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fermi import fermi, solve_mu

SPIN_SIGNS = (+1.0, -1.0)


def congruence_lowdin(S: np.ndarray) -> np.ndarray:
    """Z = S^-1/2 (symmetric), from the eigendecomposition of S."""
    lam, U = np.linalg.eigh(S)
    return (U / np.sqrt(lam)) @ U.T


def congruence_cholesky(S: np.ndarray) -> np.ndarray:
    """Z = L^-T with S = L L^T, another factor with Z^T S Z = I."""
    L = np.linalg.cholesky(S)
    return sla.solve_triangular(L, np.eye(S.shape[0]), lower=True).T


def orbital_values(per_atom: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Expand a per-atom vector to orbitals: value of orbital i = value of its atom."""
    counts = np.diff(np.asarray(offsets))
    return np.repeat(np.asarray(per_atom, dtype=np.float64), counts)


def atom_potentials(n: np.ndarray, gamma: np.ndarray, W: float):
    """u^sigma = gamma n_q + s_sigma W n_m for sigma = up, down."""
    N = gamma.shape[0]
    nq, nm = n[:N], n[N:]
    return [gamma @ nq + s * W * nm for s in SPIN_SIGNS]


def first_order_hamiltonian(u_atom: np.ndarray, S: np.ndarray, offsets) -> np.ndarray:
    """1/2 (U~ S + S U~) for per-atom potentials u."""
    ut = orbital_values(u_atom, offsets)
    return 0.5 * (ut[:, None] * S + S * ut[None, :])


def spin_hamiltonians(sysd: dict, n: np.ndarray):
    """H^sigma[n] for both spins."""
    us = atom_potentials(n, sysd["gamma"], sysd["W"])
    return [sysd["H0"] + first_order_hamiltonian(u, sysd["S"], sysd["offsets"]) for u in us]


def mulliken_populations(D: np.ndarray, S: np.ndarray, offsets) -> np.ndarray:
    """sum_{i in I} sum_j D_ij S_ji per atom I."""
    per_orbital = np.einsum("ij,ji->i", D, S)
    off = np.asarray(offsets)
    return np.array([per_orbital[off[a]:off[a + 1]].sum() for a in range(len(off) - 1)])


def expansion_point(sysd: dict, n: np.ndarray | None = None, Z: np.ndarray | None = None) -> dict:
    """Eigenbasis of both spin Hamiltonians at n (default: the system's n_ref).

    Returns Z, Q (list of two), eps (list of two), mu, kT.
    """
    if n is None:
        n = sysd["n_ref"]
    if Z is None:
        Z = congruence_lowdin(sysd["S"])
    Q, eps = [], []
    for H in spin_hamiltonians(sysd, n):
        Hperp = Z.T @ H @ Z
        Hperp = 0.5 * (Hperp + Hperp.T)
        e, q = np.linalg.eigh(Hperp)
        eps.append(e)
        Q.append(q)
    mu = solve_mu(eps, sysd["n_electrons"], sysd["kT"])
    return dict(Z=Z, Q=Q, eps=eps, mu=mu, kT=sysd["kT"])


def q_of_n(sysd: dict, n: np.ndarray, Z: np.ndarray | None = None) -> np.ndarray:
    """Ground state of the shadow functional at n, as (q, m) Mulliken vectors (length 2N)."""
    ep = expansion_point(sysd, n, Z)
    pops = []
    for Q, e in zip(ep["Q"], ep["eps"]):
        Dperp = (Q * fermi(e, ep["mu"], ep["kT"])) @ Q.T
        D = ep["Z"] @ Dperp @ ep["Z"].T
        pops.append(mulliken_populations(D, sysd["S"], sysd["offsets"]))
    return np.concatenate([pops[0] + pops[1], pops[0] - pops[1]])
