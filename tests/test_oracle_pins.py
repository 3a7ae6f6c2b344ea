"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test names what fixes the expected value: finite differences of the
full non-iterative map n -> q[n], an arbitrary-precision brute force, closed
forms, conservation laws and symmetries the mathematics implies, GMRES (a
library routine for the same Krylov minimization) and dense linear algebra.
"""

import mpmath as mp
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from oracle import fermi as ofermi
from oracle.expansion import congruence_cholesky, congruence_lowdin, expansion_point, q_of_n
from oracle.krylov import jacobian_exact, kernel_apply
from oracle.response import response, response_potentials
from synth import make_system
from tests.mp_bruteforce import response_mp


@pytest.fixture(scope="module")
def fe16():
    sysd = make_system(2, seed=16)
    return sysd, expansion_point(sysd)


@pytest.fixture(scope="module")
def fe16_stress():
    sysd = make_system(2, seed=1616, s_scale=0.9)
    return sysd, expansion_point(sysd)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


# --- Fermi factors ---------------------------------------------------------

def test_divided_differences_vs_mpmath():
    """F_ij against 50-digit (f_i - f_j)/(e_i - e_j), with ties and near-ties."""
    kT, mu = 0.25, -7.3
    gaps = [0.0, 1e-14, 1e-10, 1e-6, 1e-3, 0.05, 0.3, 1.0, 3.0, 10.0, 40.0]
    eps = [mu - 2.0]
    for g in gaps:
        eps.append(eps[0] + g)
    eps += [mu + 0.01, mu + 0.01 + 1e-12, mu + 5.0, mu - 30.0]
    eps = np.array(eps)
    F = ofermi.divided_difference_matrix(eps, mu, kT)
    with mp.workdps(50):
        def f(e):
            return 1 / (1 + mp.exp((mp.mpf(float(e)) - mp.mpf(mu)) / mp.mpf(kT)))
        worst = 0.0
        for i, ei in enumerate(eps):
            for j, ej in enumerate(eps):
                if ei == ej:
                    fi = f(ei)
                    ref = -fi * (1 - fi) / mp.mpf(kT)
                else:
                    ref = (f(ei) - f(ej)) / (mp.mpf(float(ei)) - mp.mpf(float(ej)))
                if ref != 0:
                    worst = max(worst, abs(float((mp.mpf(F[i, j]) - ref) / ref)))
    assert worst < 1e-13, worst


def test_mu_fixes_electron_count(fe16):
    sysd, ep = fe16
    n = sum(ofermi.fermi(e, ep["mu"], ep["kT"]).sum() for e in ep["eps"])
    assert abs(n - sysd["n_electrons"]) < 1e-11 * sysd["n_electrons"]


# --- response: exact derivative --------------------------------------------

def _tiny_system(seed=3):
    """2 atoms x 2 orbitals, random dense H0 and SPD S (not the Fe generator)."""
    rng = np.random.default_rng(seed)
    nb = 4
    A = rng.normal(size=(nb, nb))
    H0 = 0.5 * (A + A.T)
    B = 0.3 * rng.normal(size=(nb, nb))
    S = np.eye(nb) + 0.25 * (B + B.T) / np.abs(np.linalg.eigvalsh(B + B.T)).max()
    gamma = np.array([[0.9, 0.4], [0.4, 0.8]])
    return dict(H0=H0, S=S, gamma=gamma, W=-0.3, kT=0.2, n_electrons=3.3,
                offsets=np.array([0, 2, 4], dtype=np.int32), n_ref=np.array([0.1, -0.2, 0.7, 0.5]))


def test_response_vs_arbitrary_precision_bruteforce():
    """q1(v) equals the 50-digit central difference of the full map q[n] (both spins, mu re-solved)."""
    sysd = _tiny_system()
    ep = expansion_point(sysd)
    v = np.array([0.3, -0.8, 0.5, 0.2])
    got = response(sysd, ep, v)
    ref = response_mp(sysd["H0"], sysd["S"], sysd["gamma"], sysd["W"], list(sysd["offsets"]),
                      sysd["n_ref"], v, sysd["n_electrons"], sysd["kT"])
    assert rel(got, ref) < 1e-12, (got, ref)


def test_response_vs_finite_difference_fe16(fe16):
    """Fourth-order central difference of q[n] along v on the 16-atom system."""
    sysd, ep = fe16
    v = np.random.default_rng(5).standard_normal(2 * sysd["gamma"].shape[0])
    v /= np.linalg.norm(v)
    h = 2e-3
    n0 = sysd["n_ref"]
    q = {k: q_of_n(sysd, n0 + k * h * v, ep["Z"]) for k in (-2, -1, 1, 2)}
    fd = (-q[2] + 8 * q[1] - 8 * q[-1] + q[-2]) / (12 * h)
    got = response(sysd, ep, v)
    assert rel(got, fd) < 1e-8


def test_response_closed_form_orthogonal_diagonal():
    """S = I and diagonal H: dn_i = w_i (dmu - u_i), dmu = sum w u / sum w, per orbital."""
    rng = np.random.default_rng(11)
    N, per = 4, 3
    nb = N * per
    offsets = np.arange(0, nb + 1, per, dtype=np.int32)
    H0 = np.diag(rng.normal(0.0, 0.4, nb))
    g = rng.normal(size=(N, N))
    gamma = g @ g.T / N + np.eye(N)
    sysd = dict(H0=H0, S=np.eye(nb), gamma=gamma, W=-0.4, kT=0.25, n_electrons=5.5,
                offsets=offsets, n_ref=np.concatenate([rng.normal(0, 0.1, N), rng.normal(1.0, 0.2, N)]))
    ep = expansion_point(sysd)
    v = rng.standard_normal(2 * N)
    got = response(sysd, ep, v)
    # Independent closed form in the orbital basis: both spin Hamiltonians are diagonal.
    beta = 1.0 / sysd["kT"]
    diag_h, u_orb, w_orb = [], [], []
    for s in (1.0, -1.0):
        u_ref = gamma @ sysd["n_ref"][:N] + s * sysd["W"] * sysd["n_ref"][N:]
        diag_h.append(np.diag(H0) + np.repeat(u_ref, per))
        u_orb.append(np.repeat(gamma @ v[:N] + s * sysd["W"] * v[N:], per))
    mu = ep["mu"]
    for e in diag_h:
        f = 1.0 / (1.0 + np.exp(beta * (e - mu)))
        w_orb.append(beta * f * (1.0 - f))
    dmu = sum((w * u).sum() for w, u in zip(w_orb, u_orb)) / sum(w.sum() for w in w_orb)
    dn = [(w * (dmu - u)).reshape(N, per).sum(axis=1) for w, u in zip(w_orb, u_orb)]
    ref = np.concatenate([dn[0] + dn[1], dn[0] - dn[1]])
    assert rel(got, ref) < 1e-13


# --- response: invariants ----------------------------------------------------

def test_charge_conservation(fe16, fe16_stress):
    for sysd, ep in (fe16, fe16_stress):
        v = np.random.default_rng(2).standard_normal(2 * sysd["gamma"].shape[0])
        q1 = response(sysd, ep, v)
        N = sysd["gamma"].shape[0]
        assert abs(q1[:N].sum()) < 1e-13 * np.abs(q1).max() * N


def test_response_symmetry(fe16_stress):
    """(Gamma a)^T q1(b) = (Gamma b)^T q1(a), Gamma = diag(gamma, W I): chi is symmetric."""
    sysd, ep = fe16_stress
    N = sysd["gamma"].shape[0]
    rng = np.random.default_rng(8)
    a, b = rng.standard_normal(2 * N), rng.standard_normal(2 * N)

    def gam(x):
        return np.concatenate([sysd["gamma"] @ x[:N], sysd["W"] * x[N:]])

    lhs = gam(a) @ response(sysd, ep, b)
    rhs = gam(b) @ response(sysd, ep, a)
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), abs(rhs))


def test_potential_response_negative_semidefinite(fe16):
    """sum_sigma u^sigma . dn^sigma(u) <= 0 for any spin potentials."""
    sysd, ep = fe16
    N = sysd["gamma"].shape[0]
    rng = np.random.default_rng(9)
    for _ in range(4):
        u = [rng.standard_normal(N), rng.standard_normal(N)]
        dn = response_potentials(sysd, ep, u)
        assert u[0] @ dn[0] + u[1] @ dn[1] <= 1e-14


def test_gauge_uniform_potential(fe16):
    """u_up = u_dn = const gives H1 = c S, X = c I and no density change."""
    sysd, ep = fe16
    N = sysd["gamma"].shape[0]
    vq = np.linalg.solve(sysd["gamma"], np.full(N, 0.7))
    q1 = response(sysd, ep, np.concatenate([vq, np.zeros(N)]))
    generic = response(sysd, ep, np.random.default_rng(1).standard_normal(2 * N))
    assert np.abs(q1).max() < 1e-13 * np.abs(generic).max()


def test_unpolarized_blocks_decouple():
    """m_ref = 0, n_q = 0: H_up = H_dn, so charge and spin responses decouple."""
    sysd = make_system(2, seed=22)
    N = sysd["n_atoms"]
    sysd["n_ref"] = np.zeros(2 * N)
    ep = expansion_point(sysd)
    rng = np.random.default_rng(3)
    vq, vm = rng.standard_normal(N), rng.standard_normal(N)
    a = response(sysd, ep, np.concatenate([vq, np.zeros(N)]))
    b = response(sysd, ep, np.concatenate([np.zeros(N), vm]))
    assert np.abs(a[N:]).max() < 1e-13 * np.abs(a).max()
    assert np.abs(b[:N]).max() < 1e-13 * np.abs(b).max()


def test_spin_flip_symmetry(fe16):
    """Flipping the reference moments and v_m keeps dq and flips dm."""
    sysd, ep = fe16
    N = sysd["gamma"].shape[0]
    flipped = dict(sysd)
    flipped["n_ref"] = np.concatenate([sysd["n_ref"][:N], -sysd["n_ref"][N:]])
    epf = expansion_point(flipped, Z=ep["Z"])
    v = np.random.default_rng(4).standard_normal(2 * N)
    vf = np.concatenate([v[:N], -v[N:]])
    q1 = response(sysd, ep, v)
    q1f = response(flipped, epf, vf)
    assert rel(q1f[:N], q1[:N]) < 1e-12
    assert rel(q1f[N:], -q1[N:]) < 1e-12


def test_congruence_factor_invariance(fe16_stress):
    """Loewdin and Cholesky factors (both Z^T S Z = I) give the same response."""
    sysd, _ = fe16_stress
    Zl, Zc = congruence_lowdin(sysd["S"]), congruence_cholesky(sysd["S"])
    for Z in (Zl, Zc):
        assert np.abs(Z.T @ sysd["S"] @ Z - np.eye(len(Z))).max() < 1e-13
    v = np.random.default_rng(6).standard_normal(2 * sysd["gamma"].shape[0])
    a = response(sysd, expansion_point(sysd, Z=Zl), v)
    b = response(sysd, expansion_point(sysd, Z=Zc), v)
    assert rel(a, b) < 1e-11


def test_linearity(fe16):
    sysd, ep = fe16
    rng = np.random.default_rng(12)
    a, b = rng.standard_normal((2, 2 * sysd["gamma"].shape[0]))
    assert rel(response(sysd, ep, 2.0 * a - 3.0 * b),
               2.0 * response(sysd, ep, a) - 3.0 * response(sysd, ep, b)) < 1e-13


# --- Krylov kernel -------------------------------------------------------------

def _gmres(A, b, m):
    op = spla.LinearOperator((len(b), len(b)), matvec=A, dtype=np.float64)
    x, _ = spla.gmres(op, b, x0=np.zeros_like(b), restart=m, maxiter=1, rtol=1e-300, atol=0.0)
    return x


def test_kernel_equals_gmres(fe16):
    """m Krylov steps = GMRES(m) on (K0 J) x = K0 delta from x0 = 0 (K0 = -I and a dense K0)."""
    sysd, ep = fe16
    delta = sysd["delta"]
    n2 = len(delta)
    got = kernel_apply(sysd, ep, delta, 4)
    ref = _gmres(lambda x: -(response(sysd, ep, x) - x), -delta, 4)
    assert rel(got, ref) < 1e-10
    rng = np.random.default_rng(13)
    K0 = -np.eye(n2) + 0.05 * rng.standard_normal((n2, n2))
    got = kernel_apply(sysd, ep, delta, 5, K0)
    ref = _gmres(lambda x: K0 @ (response(sysd, ep, x) - x), K0 @ delta, 5)
    assert rel(got, ref) < 1e-10


def test_full_rank_is_inverse_jacobian(fe16):
    """m = 2N reproduces J^-1 delta; J itself agrees with finite differences of q[n]."""
    sysd, ep = fe16
    N = sysd["gamma"].shape[0]
    J = jacobian_exact(sysd, ep)
    exact = np.linalg.solve(J, sysd["delta"])
    got, parts = kernel_apply(sysd, ep, sysd["delta"], 2 * N, return_parts=True)
    assert parts["rank"] == 2 * N
    assert rel(got, exact) < 1e-11
    h = 2e-3
    for j in (0, N + 3):
        e = np.zeros(2 * N)
        e[j] = 1.0
        q = {k: q_of_n(sysd, sysd["n_ref"] + k * h * e, ep["Z"]) for k in (-2, -1, 1, 2)}
        fd = (-q[2] + 8 * q[1] - 8 * q[-1] + q[-2]) / (12 * h) - e
        assert rel(J[:, j], fd) < 1e-8


def test_exact_preconditioner_rank_one(fe16):
    """K0 = J^-1 makes K0 J = I, so one direction is exact: K delta = K0 delta."""
    sysd, ep = fe16
    K0 = np.linalg.inv(jacobian_exact(sysd, ep))
    got, parts = kernel_apply(sysd, ep, sysd["delta"], 3, K0, return_parts=True)
    assert rel(got, K0 @ sysd["delta"]) < 1e-11
    assert parts["rank"] == 1  # the second direction breaks down


def test_krylov_structure(fe16):
    sysd, ep = fe16
    _, p = kernel_apply(sysd, ep, sysd["delta"], 6, return_parts=True)
    V = p["V"]
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() < 1e-14
    assert np.linalg.eigvalsh(p["O"]).min() > 0
    # residual of the normal equations: F~^T (F~ c - f~) = 0
    ft = sysd["delta"] * -1.0
    assert np.abs(p["Ft"].T @ (p["Ft"] @ p["c"] - ft)).max() < 1e-13 * np.abs(p["Ft"]).max() ** 2


def test_breakdown_on_invariant_subspace(fe16):
    """delta along a real eigenvector of J: the Krylov space is 1-D and K delta = delta / lambda."""
    sysd, ep = fe16
    J = jacobian_exact(sysd, ep)
    lam, vecs = np.linalg.eig(J)
    k = int(np.argmin(np.abs(lam.imag) + (np.abs(lam.imag) > 0) * 1e9))
    x = vecs[:, k].real
    got, parts = kernel_apply(sysd, ep, x, 4, return_parts=True)
    assert parts["rank"] == 1
    assert rel(got, x / lam[k].real) < 1e-10


def test_zero_residual_returns_zero(fe16):
    sysd, ep = fe16
    assert not np.any(kernel_apply(sysd, ep, np.zeros(2 * sysd["gamma"].shape[0]), 4))


# --- Mulliken ------------------------------------------------------------------

def test_mulliken_total_is_trace(fe16_stress):
    """sum_I dq_I = Tr[(dD_up + dD_dn) S]; with S = I the populations are diagonal sums."""
    sysd, _ = fe16_stress
    rng = np.random.default_rng(14)
    nb = sysd["S"].shape[0]
    A, B = rng.standard_normal((2, nb, nb))
    A, B = A + A.T, B + B.T
    out = oracle.mulliken(A, B, sysd["S"], sysd["offsets"])
    N = len(sysd["offsets"]) - 1
    assert abs(out[:N].sum() - np.trace((A + B) @ sysd["S"])) < 1e-11 * np.abs(A).sum()
    assert abs(out[N:].sum() - np.trace((A - B) @ sysd["S"])) < 1e-11 * np.abs(A).sum()
    eye = oracle.mulliken(A, B, np.eye(nb), sysd["offsets"])
    dA = np.diag(A).reshape(N, -1).sum(axis=1)
    dB = np.diag(B).reshape(N, -1).sum(axis=1)
    assert np.allclose(eye, np.concatenate([dA + dB, dA - dB]), rtol=0, atol=1e-13)


def test_ground_state_population_counts_electrons(fe16):
    """Mulliken charges of the full density matrix sum to N_e."""
    sysd, _ = fe16
    q = q_of_n(sysd, sysd["n_ref"])
    N = sysd["gamma"].shape[0]
    assert abs(q[:N].sum() - sysd["n_electrons"]) < 1e-10
