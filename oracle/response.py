"""First-order response q1(v) = d q[n + lambda v] / d lambda at lambda = 0.

Test infrastructure (see the package docstring).

Sec. II.G defines the directional derivative f_v = dq[n + lambda v]/dlambda - v
and notes it can be obtained by quantum perturbation theory. Here that
derivative is written out as the exact first-order change of the Sec. II.C
construction (no finite differences):

  1. u^sigma = gamma v_q + s_sigma W v_m                  (Sec. III.A, derivative
     H1^sigma = 1/2 (U~ S + S U~)                          of the shadow energy)
  2. X^sigma = Q^T (Z^T H1^sigma Z) Q                     (perturbation in the eigenbasis)
  3. F^sigma_ij = (f_i - f_j)/(eps_i - eps_j), F_ii = f'(eps_i)
  4. dmu = sum_sigma sum_i w_i X_ii / sum_sigma sum_i w_i, w = beta f (1 - f),
     which keeps sum_sigma Tr[dD^sigma S] = 0 (fixed N_e, one shared mu)
  5. Y^sigma = F^sigma o X^sigma + dmu diag(w^sigma)      (o = elementwise)
  6. dD^sigma = Z Q Y^sigma Q^T Z^T                       (back to the AO basis)
  7. dn^sigma_I = sum_{i in I} sum_j dD^sigma_ij S_ji     (Mulliken, Sec. III.A)
  8. q1 = (dn_up + dn_dn, dn_up - dn_dn)

Every product is formed as printed, with no fusion or re-association.
"""

from __future__ import annotations

import numpy as np

from .expansion import atom_potentials, first_order_hamiltonian, mulliken_populations
from .fermi import divided_difference_matrix, fermi, fermi_complement


def response_potentials(sysd: dict, ep: dict, u_list, return_parts: bool = False):
    """Mulliken response (dn_up, dn_dn) to per-atom spin potentials (u_up, u_dn).

    This is the potential-space response chi: steps 1-7 above, starting from
    given potentials instead of from v.
    """
    S, offsets = sysd["S"], sysd["offsets"]
    Z, mu, kT = ep["Z"], ep["mu"], ep["kT"]
    beta = 1.0 / kT
    X, F, w = [], [], []
    for u, Q, e in zip(u_list, ep["Q"], ep["eps"]):
        H1 = first_order_hamiltonian(u, S, offsets)
        H1perp = Z.T @ H1 @ Z
        X.append(Q.T @ H1perp @ Q)
        F.append(divided_difference_matrix(e, mu, kT))
        w.append(beta * fermi(e, mu, kT) * fermi_complement(e, mu, kT))
    wsum = sum(wi.sum() for wi in w)
    dmu = sum((wi * np.diag(Xi)).sum() for wi, Xi in zip(w, X)) / wsum if wsum > 0 else 0.0
    dn, Ys = [], []
    for Xi, Fi, wi, Q in zip(X, F, w, ep["Q"]):
        Y = Fi * Xi + dmu * np.diag(wi)
        dD = Z @ Q @ Y @ Q.T @ Z.T
        dn.append(mulliken_populations(dD, S, offsets))
        Ys.append(Y)
    if return_parts:
        return dn, dict(X=X, F=F, w=w, Y=Ys, dmu=dmu)
    return dn


def response(sysd: dict, ep: dict, v: np.ndarray, return_parts: bool = False):
    """q1(v) as a (q, m) vector of length 2N; v is ordered (v_q, v_m)."""
    u_list = atom_potentials(np.asarray(v, dtype=np.float64), sysd["gamma"], sysd["W"])
    out = response_potentials(sysd, ep, u_list, return_parts)
    dn, parts = out if return_parts else (out, None)
    q1 = np.concatenate([dn[0] + dn[1], dn[0] - dn[1]])
    return (q1, parts) if return_parts else q1
