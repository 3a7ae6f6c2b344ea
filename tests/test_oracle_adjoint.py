"""Pins of the oracle gradient (oracle/adjoint.py) against things other than
itself: central finite differences (h = 1e-4) of the plain numpy forward
(oracle.expansion + oracle.krylov, a separate implementation), the closed
form of the full-rank case, and the input generator's gamma."""

import numpy as np
import pytest
import torch

from oracle.adjoint import U_gradient_terms, gamma_of_U, gradients
from oracle.expansion import expansion_point
from oracle.krylov import jacobian_exact, kernel_apply
from synth import make_system

H = 1e-4


@pytest.fixture(scope="module")
def fe16():
    sysd = make_system(2, seed=16)
    return sysd, gradients(sysd, 4)


def _L(sysd, m, delta=None, U=None, W=None, H0=None):
    s = dict(sysd)
    if U is not None:
        s["gamma"] = gamma_of_U(sysd["r2_bohr"], torch.tensor(U, dtype=torch.float64), sysd["hartree_ev"]).numpy()
    if W is not None:
        s["W"] = W
    if H0 is not None:
        s["H0"] = H0
    x = kernel_apply(s, expansion_point(s), sysd["delta"] if delta is None else delta, m)
    return x @ x


def test_gamma_of_U_reproduces_the_generator():
    sysd = make_system(2, seed=16)
    g = gamma_of_U(sysd["r2_bohr"], torch.tensor(sysd["U"], dtype=torch.float64), sysd["hartree_ev"]).numpy()
    assert np.abs(g - sysd["gamma"]).max() < 1e-14 * np.abs(sysd["gamma"]).max()


def test_value_matches_numpy_forward(fe16):
    sysd, g = fe16
    assert abs(g["L"] - _L(sysd, 4)) < 1e-13 * g["L"]


def test_delta_gradient_vs_finite_differences(fe16):
    sysd, g = fe16
    d = np.random.default_rng(1).standard_normal(2 * sysd["n_atoms"]) * 1e-2
    fd = (_L(sysd, 4, delta=sysd["delta"] + H * d) - _L(sysd, 4, delta=sysd["delta"] - H * d)) / (2 * H)
    assert abs(fd - g["delta"] @ d) < 1e-7 * abs(fd)


def test_U_gradient_vs_finite_differences(fe16):
    sysd, g = fe16
    hu = H * sysd["U"]
    fd = (_L(sysd, 4, U=sysd["U"] + hu) - _L(sysd, 4, U=sysd["U"] - hu)) / (2 * hu)
    assert abs(fd - g["U"]) < 1e-6 * abs(fd)


def test_W_gradient_vs_finite_differences(fe16):
    sysd, g = fe16
    hw = H * abs(sysd["W"])
    fd = (_L(sysd, 4, W=sysd["W"] + hw) - _L(sysd, 4, W=sysd["W"] - hw)) / (2 * hw)
    assert abs(fd - g["W"]) < 1e-7 * abs(fd)


def test_H0_gradient_vs_finite_differences(fe16):
    sysd, g = fe16
    E = np.random.default_rng(2).standard_normal(sysd["H0"].shape)
    E = 0.5 * (E + E.T) / np.sqrt(E.shape[0])  # spectral norm ~ 1 eV
    fd = (_L(sysd, 4, H0=sysd["H0"] + H * E) - _L(sysd, 4, H0=sysd["H0"] - H * E)) / (2 * H)
    assert abs(fd - (g["H0"] * E).sum()) < 1e-7 * abs(fd)
    assert np.abs(g["H0"] - g["H0"].T).max() < 1e-14 * np.abs(g["H0"]).max()


def test_full_rank_delta_gradient_closed_form():
    """m = 2N: K delta = J^-1 delta, so dL/d delta = 2 J^-T J^-1 delta."""
    sysd = make_system(2, seed=16)
    n2 = 2 * sysd["n_atoms"]
    g = gradients(sysd, n2)
    assert g["rank"] == n2
    J = jacobian_exact(sysd, expansion_point(sysd))
    x = np.linalg.solve(J, sysd["delta"])
    want = 2 * np.linalg.solve(J.T, x)
    assert np.linalg.norm(g["delta"] - want) < 1e-9 * np.linalg.norm(want)


def test_U_gradient_terms_sum_to_the_U_gradient(fe16):
    """The per-entry chain-rule terms through gamma add up to dL/dU (and cancel strongly)."""
    sysd, g = fe16
    terms = U_gradient_terms(sysd, 4)
    assert abs(terms.sum() - g["U"]) < 1e-10 * np.abs(terms).sum()
    assert np.abs(terms).sum() > 10 * abs(g["U"])


def test_U_gradient_terms_entry_by_entry(fe16):
    """Single terms dL/dgamma_IJ dgamma_IJ/dU, each factor by central differences on the
    plain numpy forward (one gamma entry perturbed at a time; gamma(U) from the input
    generator's formula), for the largest off-diagonal and diagonal terms."""
    sysd, _ = fe16
    m = 4
    terms = U_gradient_terms(sysd, m)
    N = terms.shape[0]
    off = np.abs(terms) * (1 - np.eye(N))
    picks = [np.unravel_index(np.argmax(off), off.shape), (int(np.argmax(np.abs(np.diag(terms)))),) * 2]
    U = float(sysd["U"])
    gp = gamma_of_U(sysd["r2_bohr"], torch.tensor(U + H, dtype=torch.float64), sysd["hartree_ev"]).numpy()
    gm = gamma_of_U(sysd["r2_bohr"], torch.tensor(U - H, dtype=torch.float64), sysd["hartree_ev"]).numpy()
    for I, J in picks:
        dg = (gp[I, J] - gm[I, J]) / (2 * H)
        hg = 1e-5 * abs(sysd["gamma"][I, J])
        Ls = []
        for sgn in (1, -1):
            s = dict(sysd)
            s["gamma"] = sysd["gamma"].copy()
            s["gamma"][I, J] += sgn * hg
            x = kernel_apply(s, expansion_point(s), sysd["delta"], m)
            Ls.append(x @ x)
        dL = (Ls[0] - Ls[1]) / (2 * hg)
        assert abs(dL * dg - terms[I, J]) < 1e-5 * abs(terms[I, J]), (I, J, dL * dg, terms[I, J])
