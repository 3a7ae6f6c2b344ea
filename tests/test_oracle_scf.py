"""Pins of the oracle's SCF acceleration and extended-Lagrangian update (CPU)."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.expansion import congruence_cholesky, expansion_point
from oracle.krylov import kernel_apply
from oracle.response import response
from oracle.scf import net_q_of_n, rms, scf, xlbomd_electrons, xlbomd_update
from synth import make_system


@pytest.fixture(scope="module")
def fe16():
    return make_system(2, seed=16)


def test_full_rank_kernel_mixer_is_newton(fe16):
    """m = 2N, no rank cut: each step is Newton's, so the residual converges quadratically."""
    n, hist = scf(fe16, fe16["n_ref"], tol=1e-13, max_iter=40, m_max=2 * fe16["n_atoms"], rank_tol=0.0,
                  switch_at=10.0)
    r = [h["rms"] for h in hist if h["mode"] == "kernel"]
    assert len(r) <= 5
    for a, b in zip(r, r[1:]):
        if b > 1e-13:
            assert b <= 10.0 * a * a, (a, b)   # r_{k+1} <= C r_k^2 with a modest C
    assert hist[-1]["mode"] == "done"


def test_scf_fixed_point(fe16):
    """The converged n satisfies q[n] = n, checked with an independent congruence factor."""
    n, hist = scf(fe16, fe16["n_ref"], tol=1e-11, max_iter=200, m_max=8, rank_tol=0.1, switch_at=10.0)
    assert hist[-1]["mode"] == "done"
    f = net_q_of_n(fe16, n, congruence_cholesky(fe16["S"])) - n
    assert rms(f) < 1e-10
    ranks = [h["rank"] for h in hist if h["mode"] == "kernel"]
    assert ranks and max(ranks) <= 8


def test_adaptive_rank_matches_gmres_residuals(fe16):
    """The chosen rank is the smallest k whose GMRES(k) residual is <= tol."""
    ep = expansion_point(fe16)
    delta = fe16["delta"]
    tol = 0.05
    _, parts = kernel_apply(fe16, ep, delta, 12, return_parts=True, tol=tol)

    def A(x):
        return -(response(fe16, ep, x) - x)

    b = -delta
    op = spla.LinearOperator((len(b), len(b)), matvec=A, dtype=np.float64)
    resid = []
    for k in range(1, 13):
        x, _ = spla.gmres(op, b, x0=np.zeros_like(b), restart=k, maxiter=1, rtol=1e-300, atol=0.0)
        resid.append(np.linalg.norm(A(x) - b) / np.linalg.norm(b))
    expect = next(k + 1 for k, r in enumerate(resid) if r <= tol)
    assert parts["rank"] == expect
    assert abs(parts["ls_residual"] - resid[expect - 1]) < 1e-8


def test_xlbomd_update_is_verlet_oscillator():
    """f = n* - n with K = -I: x = n - n* obeys x_{k+1} = (2 - kappa) x_k - x_{k-1},
    solved by x_k = A cos(k th) + B sin(k th), cos th = 1 - kappa/2."""
    kappa = 0.7
    rng = np.random.default_rng(0)
    nstar, x0 = rng.standard_normal(6), rng.standard_normal(6)
    hist = np.stack([nstar + x0, nstar + x0])          # n(t), n(t - dt)
    th = np.arccos(1.0 - kappa / 2.0)
    A, B = x0, x0 * (np.cos(th) - 1.0) / np.sin(th)
    for k in range(1, 25):
        Kf = -(nstar - hist[0])                        # K = -I applied to f = n* - n
        new = xlbomd_update(hist, Kf, kappa, 0.0, [0.0])
        hist = np.stack([new, hist[0]])
        assert np.abs(new - nstar - (A * np.cos(k * th) + B * np.sin(k * th))).max() < 1e-12


def test_xlbomd_update_dissipation_term():
    """Bookkeeping of the history rows and the dissipation sum (not a pin of the method)."""
    rng = np.random.default_rng(1)
    hist = rng.standard_normal((4, 5))
    Kf = rng.standard_normal(5)
    c = [0.5, -1.0, 0.25, 2.0]
    got = xlbomd_update(hist, Kf, 1.3, 0.01, c)
    want = 2 * hist[0] - hist[1] - 1.3 * Kf + 0.01 * (0.5 * hist[0] - hist[1] + 0.25 * hist[2] + 2 * hist[3])
    assert np.abs(got - want).max() < 1e-14


def test_xlbomd_electrons_full_rank_kernel_has_period_six():
    """Near the ground state f(n) ~ J (n - n*). With the exact kernel (full rank, K f = J^-1 f =
    n - n*) and kappa = 1 the update gives e_{k+1} = e_k - e_{k-1} for e = n - n*: a rotation by
    60 degrees. Started at rest (e_{-1} = e_0) the sequence is e_0, 0, -e_0, -e_0, 0, e_0, e_0,
    and so are the residuals f_k ~ J e_k, up to O(|e|^2) from the nonlinearity."""
    sysd = make_system(2, seed=16)
    n_star, _ = scf(sysd, sysd["n_ref"], tol=1e-12, max_iter=60, m_max=8, rank_tol=0.1, switch_at=10.0)
    e0 = 1e-5 * np.random.default_rng(5).standard_normal(n_star.size)
    res, fs, _ = xlbomd_electrons(sysd, n_star + e0, steps=7, kappa=1.0, m_max=2 * sysd["n_atoms"], rank_tol=0.0)
    f0 = fs[0]
    nf = np.linalg.norm(f0)
    for k, sign in enumerate((1, 0, -1, -1, 0, 1, 1)):
        assert np.linalg.norm(fs[k] - sign * f0) < 1e-4 * nf, (k, np.linalg.norm(fs[k] - sign * f0) / nf)
    assert abs(res[0] - rms(f0)) == 0.0
