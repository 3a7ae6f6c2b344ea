"""Preconditioned low-rank Krylov approximation of the spin-charge kernel.

Test infrastructure (see the package docstring).

Sec. II.G, in the 2N-dimensional spin-doubled space (the paper writes the
sum limits as N; the space has 2N components, so they are read as 2N):
  * the kernel is K = J^-1 with J the Jacobian of f(n) = q[n] - n;
  * with a preconditioner K0 ~ J^-1 the equation of motion uses
    (K0 J)^-1 K0 f;
  * directional derivatives f_v = q1(v) - v = J v, preconditioned
    f~_v = K0 f_v, and f~ = K0 f;
  * (K0 J)^-1 ~ sum_{k,l<=m} v_k M_kl f~_{v_l}^T with M = O^-1,
    O_kl = f~_{v_k}^T f~_{v_l} (the paper calls this Gram matrix S; it is
    named O here to avoid a clash with the overlap matrix);
  * the v_k are an orthonormal basis of the Krylov space spanned by
    f~, (K0 J) f~, (K0 J)^2 f~, ... .
Applied to f~ this is m steps of GMRES on (K0 J) x = K0 delta from x0 = 0.

Readings of points the paper leaves open: Gram-Schmidt is modified
Gram-Schmidt with one re-orthogonalization pass, v_1 = f~/||f~||; a new
direction whose norm after orthogonalization falls to <= 1e-13 of the norm
it started with ends the expansion (rank_used < m); the m x m system is
solved by Cholesky (lstsq on F~ if O is not positive definite); the
default preconditioner is K0 = -I (the scaled delta-function choice of
Sec. II.F with scale -1, since J ~ -I when the response is weak).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .response import response

BREAKDOWN_TOL = 1e-13


def _apply_k0(K0, x):
    return -x if K0 is None else K0 @ x


def _projected_solve(Fm, ftilde):
    """c minimizing ||F~ c - f~|| via the normal equations O c = F~^T f~ (Cholesky)."""
    O = Fm.T @ Fm
    rhs = Fm.T @ ftilde
    try:
        c = sla.cho_solve(sla.cho_factor(O, lower=True), rhs)
        solver = "cholesky"
    except np.linalg.LinAlgError:
        c = np.linalg.lstsq(Fm, ftilde, rcond=None)[0]
        solver = "lstsq"
    res = np.linalg.norm(Fm @ c - ftilde) / np.linalg.norm(ftilde)
    return c, O, solver, res


def kernel_apply(sysd: dict, ep: dict, delta: np.ndarray, m: int, K0: np.ndarray | None = None,
                 return_parts: bool = False, tol: float = 0.0):
    """K delta ~ (K0 J)^-1 K0 delta with a rank-m Krylov basis.

    tol > 0 chooses the rank adaptively: after each new direction the projected
    problem is solved and the expansion stops once ||F~ c - f~|| / ||f~|| <= tol
    (at most m directions). Sec. III.C uses a few ranks per SCF step chosen
    adaptively; this residual criterion is our reading.
    """
    delta = np.asarray(delta, dtype=np.float64)
    ftilde = _apply_k0(K0, delta)
    nrm0 = np.linalg.norm(ftilde)
    V, Ft, Q1 = [], [], []
    if nrm0 == 0.0:
        out = np.zeros_like(delta)
        return (out, dict(V=V, Ft=Ft, q1=Q1, rank=0, c=np.zeros(0), O=np.zeros((0, 0)),
                          ls_residual=0.0)) if return_parts else out
    r = ftilde
    for k in range(m):
        w = r.copy()
        start = np.linalg.norm(w)
        for _ in range(2):  # MGS, then one re-orthogonalization pass
            for vj in V:
                w = w - (vj @ w) * vj
        nw = np.linalg.norm(w)
        if nw <= BREAKDOWN_TOL * start:
            break
        vk = w / nw
        q1 = response(sysd, ep, vk)
        fv = q1 - vk                      # f_v = J v
        ftk = _apply_k0(K0, fv)           # f~_v = K0 J v
        V.append(vk)
        Ft.append(ftk)
        Q1.append(q1)
        r = ftk
        if tol > 0.0 and len(V) < m:
            if _projected_solve(np.array(Ft).T, ftilde)[3] <= tol:
                break
    rank = len(V)
    Vm = np.array(V).T                    # 2N x rank
    Fm = np.array(Ft).T
    c, O, solver, res = _projected_solve(Fm, ftilde)
    out = Vm @ c
    if return_parts:
        return out, dict(V=Vm, Ft=Fm, q1=np.array(Q1).T, rank=rank, c=c, O=O, solver=solver,
                         ls_residual=res)
    return out


def jacobian_exact(sysd: dict, ep: dict) -> np.ndarray:
    """J = [q1(e_j) - e_j]_j, the full 2N x 2N Jacobian of f(n) = q[n] - n."""
    n2 = 2 * sysd["gamma"].shape[0]
    J = np.empty((n2, n2))
    for j in range(n2):
        e = np.zeros(n2)
        e[j] = 1.0
        J[:, j] = response(sysd, ep, e) - e
    return J
