"""Differentiation form on the GPU: the hand-written reverse pass of the HIP
library (krylov_kernel_adjoint behind torch.autograd) against the oracle
gradient (torch.autograd through the plain CPU forward, oracle/adjoint.py)
and against central finite differences (h = 1e-4) of the oracle's forward,
for L = ||K delta||^2 with respect to delta, U, W and H0.
"""

import json
import os

import numpy as np
import pytest

from tests.gpu_helpers import DEV, handle_from_expansion, rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.adjoint import U_gradient_scale, gradients  # noqa: E402
from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from paper_2303_03529_amd.autograd import KernelSystem, kernel_from_parameters  # noqa: E402
from paper_2303_03529_amd.krylov import KK_FP64, KK_MIXED_BF16, KK_MIXED_F16  # noqa: E402
from synth import gradient_direction, make_system, symmetric_direction  # noqa: E402

TOL = 1e-10
GOLD432 = os.path.join(os.path.dirname(__file__), "golden", "fe432grad_oracle.json")
GOLD1024 = os.path.join(os.path.dirname(__file__), "golden", "fe1024fd_oracle.json")


def gpu_gradients(sysd, m, K0=None, precision=0):
    """L and dL/d(delta, U, W, H0) through KrylovKernel on the device."""
    ks = KernelSystem(sysd, device=DEV, precision=precision)
    try:
        d = t(sysd["delta"]).requires_grad_(True)
        U = torch.tensor(sysd["U"], dtype=torch.float64, device=DEV, requires_grad=True)
        W = torch.tensor(sysd["W"], dtype=torch.float64, device=DEV, requires_grad=True)
        H0 = t(sysd["H0"]).requires_grad_(True)
        if K0 is not None:
            raise NotImplementedError
        x = kernel_from_parameters(ks, d, U, W, H0, m)
        L = x @ x
        gd, gu, gw, gh = torch.autograd.grad(L, [d, U, W, H0])
        return dict(L=float(L.detach()), delta=gd.cpu().numpy(), U=float(gu), W=float(gw), H0=gh.cpu().numpy())
    finally:
        ks.close()


def compare(got, ref, tol=TOL, U_scale=None):
    """Relative errors; dL/dU relative to U_scale (the sum of its terms' magnitudes) if given."""
    errs = {
        "L": abs(got["L"] - ref["L"]) / abs(ref["L"]),
        "delta": rel(got["delta"], ref["delta"]),
        "U": abs(got["U"] - ref["U"]) / (U_scale if U_scale is not None else abs(ref["U"])),
        "W": abs(got["W"] - ref["W"]) / abs(ref["W"]),
        "H0": rel(got["H0"], ref["H0"]),
    }
    print("adjoint vs oracle gradient:", {k: f"{v:.1e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < tol, (k, v)


@pytest.mark.parametrize("m", [4, 8])
def test_adjoint_fe16_matches_oracle_gradient(m):
    sysd = make_system(2, seed=16)
    compare(gpu_gradients(sysd, m), gradients(sysd, m))


def test_adjoint_fe128_matches_oracle_gradient():
    sysd = make_system(4, seed=128)
    compare(gpu_gradients(sysd, 8), gradients(sysd, 8))


@pytest.mark.parametrize("precision", [KK_MIXED_F16, KK_MIXED_BF16], ids=["split_f16", "bf16"])
def test_adjoint_split_forward_fe128(precision):
    """Split-precision forward, FP64 reverse sweep: the gradient of the split forward map,
    within the split form's 1e-6 of the oracle gradient. dL/dU is a sum whose terms cancel
    ~260-fold here; its error is bounded against their size (the plain relative error, up to
    1e-6 times that ratio, is printed too)."""
    sysd = make_system(4, seed=128)
    scale = U_gradient_scale(sysd, 8)
    got, ref = gpu_gradients(sysd, 8, precision=precision), gradients(sysd, 8)
    u_plain = abs(got["U"] - ref["U"]) / abs(ref["U"])
    print(f"split fe128 ({precision}): dL/dU plain relative error {u_plain:.1e}, "
          f"terms/result {scale / abs(ref['U']):.0f}", flush=True)
    compare(got, ref, tol=1e-6, U_scale=scale)
    assert u_plain < 1e-6 * scale / abs(ref["U"])


def test_adjoint_ragged_cluster_matches_oracle_gradient():
    sysd = make_system(n_atoms=37, seed=10_037)
    compare(gpu_gradients(sysd, 6), gradients(sysd, 6))


def test_adjoint_reuse_equals_recompute():
    """reuse_forward=1 after krylov_kernel_apply gives the same gradients as a fresh expansion."""
    sysd = make_system(2, seed=16)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep)
    try:
        d = t(sysd["delta"])
        x, _ = h.krylov_kernel_apply(d, 6)
        a = h.krylov_kernel_adjoint(d, 6, 2 * x, reuse_forward=True)
        b = h.krylov_kernel_adjoint(d, 6, 2 * x, reuse_forward=False, want_Kdelta=True)
        assert rel(b["Kdelta"].cpu().numpy(), x.cpu().numpy()) < 1e-15
        for k in ("delta", "gamma", "H_up", "H_dn"):
            assert rel(a[k].cpu().numpy(), b[k].cpu().numpy()) < 1e-14, k
        assert abs(float(a["W"]) - float(b["W"])) <= 1e-14 * abs(float(b["W"]))
        with pytest.raises(Exception):
            h.krylov_kernel_adjoint(d, 5, 2 * x, reuse_forward=True)  # m differs from the last call
    finally:
        h.close()


def test_adjoint_dense_preconditioner_delta_gradient():
    """K0 dense (the chain through K0^T): dL/d delta against the oracle gradient with
    the same K0, and against a central difference of the oracle's forward (whose
    O(h^2) error is ~1e-6 here: L is far from quadratic in delta along this direction)."""
    sysd = make_system(2, seed=16)
    ep = expansion_point(sysd)
    n2 = 2 * sysd["n_atoms"]
    R = np.random.default_rng(7).standard_normal((n2, n2)) / np.sqrt(n2)
    K0 = -(np.eye(n2) + 0.2 * R)
    h = handle_from_expansion(sysd, ep)
    try:
        d, k0 = t(sysd["delta"]), t(K0)
        x, _ = h.krylov_kernel_apply(d, 6, K0=k0)
        g = h.krylov_kernel_adjoint(d, 6, 2 * x, K0=k0, reuse_forward=True)
    finally:
        h.close()
    dd = np.random.default_rng(8).standard_normal(n2) * 1e-2
    hh = 1e-4

    def L(delta):
        y = kernel_apply(sysd, ep, delta, 6, K0=K0)
        return y @ y
    fd = (L(sysd["delta"] + hh * dd) - L(sysd["delta"] - hh * dd)) / (2 * hh)
    an = g["delta"].cpu().numpy() @ dd
    ref = gradients(sysd, 6, K0=K0)["delta"]
    err = rel(g["delta"].cpu().numpy(), ref)
    print(f"dense K0: FD {fd:.12e} adjoint {an:.12e}; vs oracle gradient {err:.1e}")
    assert err < TOL
    assert abs(fd - an) < 2e-6 * abs(fd)


def test_adjoint_exact_degeneracies():
    """S = I and a diagonal H with repeated levels (every d, p level degenerate):
    dL/dH0 along a random symmetric direction against central differences of the
    oracle, which needs the near-degenerate pair path of the reverse pass."""
    N, per = 6, 9
    nb = N * per
    onsite = np.tile([-4.0, 2.0, 2.0, 2.0, -8.5, -8.5, -8.5, -8.5, -8.5], N)
    g = np.random.default_rng(4).normal(size=(N, N))
    sysd = dict(H0=np.diag(onsite), S=np.eye(nb), gamma=g @ g.T / N + np.eye(N), W=-0.4,
                kT=0.25, n_electrons=8.0 * N, offsets=np.arange(0, nb + 1, per, dtype=np.int32),
                n_ref=np.concatenate([np.zeros(N), np.full(N, 0.5)]), n_atoms=N,
                delta=np.random.default_rng(6).normal(0, 0.01, 2 * N))
    m = 4
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep)
    try:
        x, _ = h.krylov_kernel_apply(t(sysd["delta"]), m)
        gr = h.krylov_kernel_adjoint(t(sysd["delta"]), m, 2 * x, reuse_forward=True)
    finally:
        h.close()
    E = np.random.default_rng(9).standard_normal((nb, nb))
    E = 0.5 * (E + E.T) / np.sqrt(nb)
    hh = 1e-4

    def L(H0):
        s = dict(sysd, H0=H0)
        y = kernel_apply(s, expansion_point(s), sysd["delta"], m)
        return y @ y
    fd = (L(sysd["H0"] + hh * E) - L(sysd["H0"] - hh * E)) / (2 * hh)
    an = float(((gr["H_up"] + gr["H_dn"]).cpu().numpy() * E).sum())
    print(f"degenerate levels: FD {fd:.12e} adjoint {an:.12e}")
    assert abs(fd - an) < 1e-6 * abs(fd)


def _direction_dot(g, d):
    """Directional derivative sum over (delta, U, W, H0) of gradient times direction."""
    return float(g["delta"] @ d["delta"] + g["U"] * d["U"] + g["W"] * d["W"] + (g["H0"] * d["H0"]).sum())


@pytest.mark.parametrize("precision,tol", [(KK_FP64, 1e-6), (KK_MIXED_F16, 1e-5), (KK_MIXED_BF16, 1e-5)],
                         ids=["fp64", "split_f16", "bf16"])
def test_adjoint_fe1024_vs_oracle_finite_difference(precision, tol):
    """1024-atom bcc Fe, m = 12 (the differentiation workload): the adjoint's directional
    derivative along d = synth.gradient_direction(sysd, 11) in (delta, U, W, H0) against the
    oracle's central difference (h = 1e-4) of its own plain forward, stored by
    make_oracle_golden.py (fe1024fd). The bound covers the difference's O(h^2) truncation
    (1e-6; the 16-atom oracle pins put it below 1e-7) and, for the split forwards, the
    gradient of the split map (1e-5). L itself: 1e-10 (FP64), 2e-6 (split)."""
    if not os.path.exists(GOLD1024):
        pytest.skip("fe1024fd golden not generated")
    gold = json.load(open(GOLD1024))
    sysd = make_system(gold["cells"], seed=gold["seed"])
    d = gradient_direction(sysd, gold["dir_seed"])
    g = gpu_gradients(sysd, gold["rank"], precision=precision)
    an = _direction_dot(g, d)
    e_fd = abs(an - gold["fd"]) / abs(gold["fd"])
    e_L = abs(g["L"] - gold["L"]) / gold["L"]
    print(f"1024 atoms, precision {precision}: adjoint {an:.12e}, oracle FD {gold['fd']:.12e}, rel {e_fd:.1e}; "
          f"L rel {e_L:.1e}", flush=True)
    assert e_L < (1e-10 if precision == KK_FP64 else 2e-6)
    assert e_fd < tol


@pytest.mark.parametrize("precision", [KK_FP64, KK_MIXED_F16, KK_MIXED_BF16], ids=["fp64", "split_f16", "bf16"])
def test_adjoint_fe432_vs_oracle_gradient(precision):
    """432-atom bcc Fe, m = 8: every gradient against the oracle gradient (torch.autograd through
    the plain CPU forward, stored by make_oracle_golden.py as fe432grad): dL/d delta, dL/dU,
    dL/dW, and dL/dH0 through its diagonal, Frobenius norm and projections on 8 seeded
    symmetric directions. The library is prepared from its own device eigensolve.
    Bounds: 1e-10 (FP64), 1e-6 (split forwards, FP64 reverse sweep). dL/dU is a sum whose
    terms cancel (their magnitudes add up to U_term_scale, ~20 |dL/dU| here): its error is
    bounded by tol x U_term_scale, i.e. a plain relative error up to tol x that ratio; both
    numbers are printed."""
    gold = json.load(open(GOLD432))
    sysd = make_system(gold["cells"], seed=gold["seed"])
    g = gpu_gradients(sysd, gold["rank"], precision=precision)
    tol = TOL if precision == KK_FP64 else 1e-6
    nb = sysd["n_basis"]
    proj = np.array([(g["H0"] * symmetric_direction(nb, gold["h0_dir_seed"] + k)).sum()
                     for k in range(len(gold["H0_proj"]))])
    errs = {
        "L": abs(g["L"] - gold["L"]) / gold["L"],
        "delta": rel(g["delta"], gold["delta"]),
        "W": abs(g["W"] - gold["W"]) / abs(gold["W"]),
        "H0_diag": rel(np.diag(g["H0"]), gold["H0_diag"]),
        "H0_proj": rel(proj, gold["H0_proj"]),
        "H0_fro": abs(np.linalg.norm(g["H0"]) - gold["H0_fro"]) / gold["H0_fro"],
        "U_vs_terms": abs(g["U"] - gold["U"]) / gold["U_term_scale"],
    }
    u_plain = abs(g["U"] - gold["U"]) / abs(gold["U"])
    ratio = gold["U_term_scale"] / abs(gold["U"])
    print(f"432 atoms, precision {precision}: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items())
          + f"; dL/dU plain relative {u_plain:.1e} (terms/result {ratio:.0f})", flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)
    assert u_plain < tol * ratio


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6), (2, 1e-6)], ids=["fp64", "split", "bf16"])
def test_adjoint_without_H_gradients(precision, tol):
    """H_bar = NULL: only dL/d delta, dL/d gamma and dL/dW, from one transposed response per
    direction in the handle's precision; against the oracle gradient (delta) and the full
    FP64 reverse pass (gamma, W)."""
    sysd = make_system(4, seed=128)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, precision)
    h64 = handle_from_expansion(sysd, ep, 0)
    try:
        d = t(sysd["delta"])
        x, _ = h.krylov_kernel_apply(d, 8)
        g = h.krylov_kernel_adjoint(d, 8, 2 * x, reuse_forward=True, want_H=False)
        assert g["H_up"] is None and g["H_dn"] is None
        x64, _ = h64.krylov_kernel_apply(d, 8)
        full = h64.krylov_kernel_adjoint(d, 8, 2 * x64, reuse_forward=True)
    finally:
        h.close()
        h64.close()
    ref = gradients(sysd, 8)
    err_d = rel(g["delta"].cpu().numpy(), ref["delta"])
    err_g = rel(g["gamma"].cpu().numpy(), full["gamma"].cpu().numpy())
    err_w = abs(float(g["W"]) - float(full["W"])) / abs(float(full["W"]))
    print(f"without H: delta {err_d:.1e}, gamma {err_g:.1e}, W {err_w:.1e}")
    assert err_d < tol and err_g < tol and err_w < tol
