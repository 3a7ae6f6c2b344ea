"""Edge cases of the HIP path against the oracle: the smallest system (one
atom), atoms with different orbital counts, the largest rank, a batch of one,
the reverse pass after a breakdown, and sizes beyond the supported range."""

import numpy as np
import pytest

from tests.gpu_helpers import handle_from_expansion, rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.adjoint import gradients  # noqa: E402
from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from oracle.response import response  # noqa: E402
from paper_2303_03529_amd import krylov  # noqa: E402
from synth import krylov_vectors, make_system  # noqa: E402

TOL = {krylov.KK_FP64: 1e-10, krylov.KK_MIXED_F16: 1e-6, krylov.KK_MIXED_BF16: 1e-6}


def ragged_orbitals(sysd, counts):
    """The same system keeping only the first counts[I] orbitals of atom I (1..9)."""
    off = sysd["offsets"]
    keep = np.concatenate([np.arange(off[a], off[a] + c) for a, c in enumerate(counts)])
    out = dict(sysd)
    out["H0"] = sysd["H0"][np.ix_(keep, keep)]
    out["S"] = sysd["S"][np.ix_(keep, keep)]
    out["offsets"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    out["n_basis"] = int(len(keep))
    out["n_electrons"] = float(0.9 * len(keep))  # keep 0 < N_e < 2 Nb with partial filling
    return out


@pytest.mark.parametrize("precision", [krylov.KK_FP64, krylov.KK_MIXED_F16, krylov.KK_MIXED_BF16],
                         ids=["fp64", "split", "bf16"])
def test_single_atom(precision):
    sysd = make_system(n_atoms=1, seed=10_001)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, precision)
    try:
        v = krylov_vectors(1, 2, 5)
        q = h.density_response_batch(t(v)).cpu().numpy()
        for i in range(2):
            assert rel(q[i], response(sysd, ep, v[i])) < TOL[precision]
        kd, info = h.krylov_kernel_apply(t(sysd["delta"]), 2)
        assert info.rank_used <= 2
        assert rel(kd.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 2)) < TOL[precision]
    finally:
        h.close()


@pytest.mark.parametrize("precision", [krylov.KK_FP64, krylov.KK_MIXED_F16, krylov.KK_MIXED_BF16],
                         ids=["fp64", "split", "bf16"])
def test_atoms_with_different_orbital_counts(precision):
    base = make_system(2, seed=16)
    counts = np.array([1, 4, 9, 9, 4, 1, 9, 2, 9, 9, 3, 9, 5, 9, 9, 7])
    sysd = ragged_orbitals(base, counts)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, precision)
    try:
        v = krylov_vectors(16, 3, 6)
        q = h.density_response_batch(t(v)).cpu().numpy()
        for i in range(3):
            assert rel(q[i], response(sysd, ep, v[i])) < TOL[precision]
        kd, _ = h.krylov_kernel_apply(t(sysd["delta"]), 6)
        assert rel(kd.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 6)) < TOL[precision]
    finally:
        h.close()


def test_largest_rank():
    """m = 64 (the library's maximum) on a 37-atom cluster (2N = 74)."""
    sysd = make_system(n_atoms=37, seed=10_037)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep)
    try:
        kd, info = h.krylov_kernel_apply(t(sysd["delta"]), 64)
        ref, parts = kernel_apply(sysd, ep, sysd["delta"], 64, return_parts=True)
        cond = np.linalg.cond(parts["O"])
        err = rel(kd.cpu().numpy(), ref)
        print(f"m = 64: rank {info.rank_used}, cond(O) {cond:.1e}, error {err:.1e}")
        assert info.rank_used == parts["rank"]
        assert err < max(1e-10, 1e-15 * cond)
        with pytest.raises(krylov.KKError):
            h.krylov_kernel_apply(t(sysd["delta"]), 65)
    finally:
        h.close()


def test_batch_of_one_system():
    from paper_2303_03529_amd.caller_setup import DeviceSystem
    sysd = make_system(n_atoms=29, seed=10_029)
    e = DeviceSystem(sysd, "cuda").expansion()
    b = krylov.Batch().prepare([dict(offsets=sysd["offsets"], S=e["S"], Z=e["Z"], Q_up=e["Q_up"], Q_dn=e["Q_dn"],
                                     eps_up=e["eps_up"], eps_dn=e["eps_dn"], gamma=e["gamma"], W=sysd["W"],
                                     kT=sysd["kT"], n_electrons=sysd["n_electrons"])])
    try:
        outs, infos = b.krylov_kernel_apply([t(sysd["delta"])], 5)
        ref = kernel_apply(sysd, expansion_point(sysd), sysd["delta"], 5)
        assert infos[0].rank_used == 5
        assert rel(outs[0].cpu().numpy(), ref) < 1e-10
    finally:
        b.close()


def test_adjoint_after_breakdown():
    """delta in a 2-dimensional invariant subspace of K0 J: the expansion stops at
    rank 2 (KK_BREAKDOWN) and the reverse pass differentiates the rank-2 map,
    which the oracle gradient at m = 2 gives."""
    sysd = make_system(2, seed=16)
    ep = expansion_point(sysd)
    from oracle.krylov import jacobian_exact
    J = jacobian_exact(sysd, ep)
    lam, vec = np.linalg.eig(-J)
    real = np.argsort(np.abs(lam.imag))[:2]
    delta = np.real(vec[:, real[0]]) * 0.01 + np.real(vec[:, real[1]]) * 0.02
    h = handle_from_expansion(sysd, ep)
    try:
        x, info = h.krylov_kernel_apply(t(delta), 6)
        assert info.rank_used == 2 and info.status == krylov.KK_BREAKDOWN
        g = h.krylov_kernel_adjoint(t(delta), 6, 2 * x, reuse_forward=True)
        assert g["info"].rank_used == 2
        ref = gradients(sysd, 2, delta=delta)
        assert rel(g["delta"].cpu().numpy(), ref["delta"]) < 1e-8
    finally:
        h.close()


def test_prepare_rejects_out_of_range_sizes():
    """kk_prepare checks the sizes before touching any array: more than 65536 basis
    functions or 4096 atoms is KK_EINVAL with a message, and the same handle then
    prepares a valid system and matches the oracle."""
    import ctypes
    dummy = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    h = krylov.Handle()
    try:
        for n_atoms, nb in ((1, 70000), (4097, 4097 * 9)):
            off = np.linspace(0, nb, n_atoms + 1).astype(np.int32)
            rc = krylov.LIB.kk_prepare(h._h, n_atoms, off.ctypes.data_as(ctypes.c_void_p), nb, p, p, p, p, p, p, p,
                                       -0.4, 0.25, 8.0, krylov.KK_FP64)
            assert rc == krylov.KK_EINVAL
            assert ("65536" if nb == 70000 else "4096") in krylov.last_error()
        sysd = make_system(2, seed=16)
        ep = expansion_point(sysd)
        h.prepare(sysd["offsets"], t(sysd["S"]), t(ep["Z"]), t(ep["Q"][0]), t(ep["Q"][1]), t(ep["eps"][0]),
                  t(ep["eps"][1]), t(sysd["gamma"]), sysd["W"], sysd["kT"], sysd["n_electrons"], krylov.KK_FP64)
        x, _ = h.krylov_kernel_apply(t(sysd["delta"]), 4)
        assert rel(x.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 4)) < 1e-10
    finally:
        h.close()


@pytest.mark.parametrize("precision", [krylov.KK_FP64, krylov.KK_MIXED_F16, krylov.KK_MIXED_BF16],
                         ids=["fp64", "split", "bf16"])
def test_ragged_atoms_across_tile_rows(precision):
    """54 atoms with 1-9 orbitals each (Nb = 325, padded 384): atoms 22 and 42 straddle the
    128-row tiles of the products, so their Mulliken sums gather partial rows of two tiles.
    Three responses and the rank-6 kernel against the oracle."""
    base = make_system(3, seed=54)
    pattern = [1, 4, 9, 9, 4, 1, 9, 2, 9, 9, 3, 9, 5, 9, 9, 7]
    counts = np.array([pattern[i % len(pattern)] for i in range(base["n_atoms"])])
    sysd = ragged_orbitals(base, counts)
    off = sysd["offsets"]
    straddling = [a for a in range(len(counts)) if off[a] // 128 != (off[a + 1] - 1) // 128]
    assert straddling == [22, 42] and sysd["n_basis"] == 325
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, precision)
    try:
        v = krylov_vectors(base["n_atoms"], 3, 7)
        q = h.density_response_batch(t(v)).cpu().numpy()
        for i in range(3):
            assert rel(q[i], response(sysd, ep, v[i])) < TOL[precision]
        kd, info = h.krylov_kernel_apply(t(sysd["delta"]), 6)
        err = rel(kd.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 6))
        print(f"ragged 54 atoms (Nb {sysd['n_basis']}), precision {precision}: kernel {err:.2e}, "
              f"rank {info.rank_used}", flush=True)
        assert err < TOL[precision]
    finally:
        h.close()
