"""Differentiation form on the GPU: the hand-written reverse pass of the HIP
library (krylov_kernel_adjoint behind torch.autograd) against the oracle
gradient (torch.autograd through the plain CPU forward, oracle/adjoint.py)
and against central finite differences (h = 1e-4) of the oracle's forward,
for L = ||K delta||^2 with respect to delta, U, W and H0.
"""

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
from synth import make_system  # noqa: E402

TOL = 1e-10


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


def test_adjoint_split_forward_fe128():
    """Split-precision forward (KK_MIXED_F16), FP64 reverse sweep: the gradient of the
    split forward map, within the split form's 1e-6 of the oracle gradient. dL/dU is a
    sum whose terms cancel ~260-fold here; its error is measured against their size."""
    sysd = make_system(4, seed=128)
    scale = U_gradient_scale(sysd, 8)
    compare(gpu_gradients(sysd, 8, precision=1), gradients(sysd, 8), tol=1e-6, U_scale=scale)


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


def test_adjoint_fullsize_directional_derivative():
    """1024-atom bcc Fe, m = 12 (the differentiation workload): the gradient
    along a random direction of (delta, U, W, H0) against a central difference
    (h = 1e-4) of the device forward itself, each side of which re-solves the
    eigenproblem."""
    sysd = make_system(8, seed=1024)
    m = 12
    ks = KernelSystem(sysd, device=DEV)
    try:
        d = t(sysd["delta"]).requires_grad_(True)
        U = torch.tensor(sysd["U"], dtype=torch.float64, device=DEV, requires_grad=True)
        W = torch.tensor(sysd["W"], dtype=torch.float64, device=DEV, requires_grad=True)
        H0 = t(sysd["H0"]).requires_grad_(True)
        x = kernel_from_parameters(ks, d, U, W, H0, m)
        L = x @ x
        gd, gu, gw, gh = torch.autograd.grad(L, [d, U, W, H0])
        rng = np.random.default_rng(11)
        nb = sysd["n_basis"]
        dd = t(rng.standard_normal(2 * sysd["n_atoms"]) * 1e-2)
        E = rng.standard_normal((nb, nb))
        dH = t(0.5 * (E + E.T) / np.sqrt(nb))
        du, dw = 0.1 * sysd["U"], 0.1 * abs(sysd["W"])
        an = float(gd @ dd + gu * du + gw * dw + (gh * dH).sum())
        hh = 1e-4

        def Lat(s):
            with torch.no_grad():
                y = kernel_from_parameters(ks, d.detach() + s * dd, U.detach() + s * du, W.detach() + s * dw,
                                           H0.detach() + s * dH, m)
                return float(y @ y)
        fd = (Lat(hh) - Lat(-hh)) / (2 * hh)
        print(f"1024 atoms: FD {fd:.12e} adjoint {an:.12e} rel {abs(fd - an) / abs(fd):.1e}")
        assert abs(fd - an) < 1e-5 * abs(fd)
    finally:
        ks.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)], ids=["fp64", "split"])
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
