"""Kernel-accelerated SCF and the extended-Lagrangian electronic update.

Test infrastructure (see the package docstring).

Sec. III.C: a quasi-Newton SCF, n_new = n_old - K (q[n_old] - n_old), with K
the preconditioned low-rank Krylov kernel of Sec. II.G evaluated at the
current n, using a few ranks per step chosen adaptively; a plain linear mixer
n_new = n_old + a (q[n_old] - n_old) (a = 0.06 in the paper's Fe example) is the
baseline, and the kernel mixer starts once the charge error of the linear
mixer is below 0.05. The error measure is the root mean square of the
residual q[n] - n.

Sec. II.F: n(t+dt) = 2 n(t) - n(t-dt) + dt^2 n''(t) + alpha sum_k c_k n(t - k dt)
with n'' = -omega^2 K (q[n] - n); with kappa = dt^2 omega^2 the update is
2 n - n_prev - kappa K f + alpha sum_k c_k n(t - k dt). The coefficients come
from earlier work and are inputs.
"""

from __future__ import annotations

import numpy as np

from .expansion import expansion_point, q_of_n
from .krylov import kernel_apply


def rms(x) -> float:
    return float(np.sqrt(np.mean(np.asarray(x) ** 2)))


def net_q_of_n(sysd: dict, n: np.ndarray, Z=None) -> np.ndarray:
    """q[n] with the neutral-atom reference removed from the charges (Sec. III.A:
    Mulliken charges of D - D0); the moments carry no reference."""
    q = q_of_n(sysd, n, Z)
    N = len(sysd["valence"])
    q[:N] -= sysd["valence"]
    return q


def scf(sysd: dict, n0: np.ndarray, mixer: str = "kernel", tol: float = 1e-8, max_iter: int = 100,
        m_max: int = 8, rank_tol: float = 0.1, linear_coeff: float = 0.06, switch_at: float = 0.05,
        K0=None, Z=None):
    """Returns (n, history) with history a list of dicts (rms residual, rank, mode)."""
    n = np.array(n0, dtype=np.float64)
    hist = []
    for _ in range(max_iter):
        ep = expansion_point(sysd, n, Z)
        f = net_q_of_n(sysd, n, ep["Z"]) - n
        err = rms(f)
        if err <= tol:
            hist.append(dict(rms=err, rank=0, mode="done"))
            break
        if mixer == "linear" or err > switch_at:
            hist.append(dict(rms=err, rank=0, mode="linear"))
            n = n + linear_coeff * f
            continue
        Kf, parts = kernel_apply(sysd, ep, f, m_max, K0, return_parts=True, tol=rank_tol)
        hist.append(dict(rms=err, rank=parts["rank"], mode="kernel"))
        n = n - Kf
    return n, hist


def xlbomd_update(n_hist: np.ndarray, Kf: np.ndarray, kappa: float, alpha: float, c) -> np.ndarray:
    """n(t+dt) from rows n_hist[k] = n(t - k dt), k = 0..k_max."""
    n_hist = np.asarray(n_hist, dtype=np.float64)
    prev = n_hist[1] if len(n_hist) > 1 else n_hist[0]
    diss = sum(ck * n_hist[k] for k, ck in enumerate(c))
    return 2.0 * n_hist[0] - prev - kappa * np.asarray(Kf) + alpha * diss


def xlbomd_electrons(sysd: dict, n_start: np.ndarray, steps: int, kappa: float, alpha: float = 0.0, c=(1.0,),
                     m_max: int = 4, rank_tol: float = 0.1, K0=None):
    """Extended-Lagrangian propagation of n at fixed nuclei (Sec. II.F with the kernel of II.G).

    The history starts with every row n(t - k dt) = n_start. Each step forms the
    residual f = q[n(t)] - n(t) at a fresh expansion point, applies the
    adaptive-rank kernel (as in the SCF above) and takes the update
    n(t+dt) = 2 n(t) - n(t-dt) - kappa K f + alpha sum_k c_k n(t - k dt).
    Returns (rms residual per step, residual vectors per step, final n).
    """
    kmax = max(len(c) - 1, 1)
    hist = np.tile(np.asarray(n_start, dtype=np.float64), (kmax + 1, 1))
    cc = np.zeros(kmax + 1)
    cc[: len(c)] = c
    res, fs = [], []
    for _ in range(steps):
        n = hist[0]
        ep = expansion_point(sysd, n)
        f = net_q_of_n(sysd, n, ep["Z"]) - n
        res.append(rms(f))
        fs.append(f)
        Kf = kernel_apply(sysd, ep, f, m_max, K0, tol=rank_tol)
        new = xlbomd_update(hist, Kf, kappa, alpha, cc)
        hist = np.vstack([new[None, :], hist[:-1]])
    return res, fs, hist[0]
