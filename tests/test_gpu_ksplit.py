"""K-split and stream-K transforms of small single systems against the FP64 oracle, on
open clusters in all three precisions: 56 atoms (Nb = 504, padded 512: two chunks of 256
rows on 64 x 64 tiles in every form) and 113 atoms (Nb = 1017, padded 1024, contraction
1024: two chunks of 512 rows on 128 x 128 tiles); and 170 atoms (Nb = 1530, padded 1536), where the split forms' products
run stream-K (288 tiles for 256 workgroups, two segments per tile at most; the batched
responses' launch of five directions too) and FP64 runs unsplit on 64 x 64 tiles; and 140
atoms (Nb = 1260, padded 1280), where FP64 runs unsplit on 128 x 128 tiles (200 workgroups,
one per CU) and the split forms on theirs, unsplit; and 250 atoms (Nb = 2250, padded 2304),
where FP64 runs 128 x 128 tiles with the full-tile forward in three rounds of workgroups (the
largest padded size the small-system rules decide) and the split forms three rounds of theirs.

Checked: five responses in one call (the workspace holds two directions at a time
with four chunks, so the call runs in three batches), each against the oracle's
response, and the rank-6 kernel against the oracle's kernel. Bounds: 1e-10 (FP64) and
1e-6 (split forms), relative 2-norm per output.
"""

import numpy as np
import pytest

from tests.gpu_helpers import handle_from_expansion, rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from oracle.response import response  # noqa: E402
from paper_2303_03529_amd import krylov  # noqa: E402
from synth import make_system  # noqa: E402

TOL = {krylov.KK_FP64: 1e-10, krylov.KK_MIXED_F16: 1e-6, krylov.KK_MIXED_BF16: 1e-6}
PRECISIONS = [krylov.KK_FP64, krylov.KK_MIXED_F16, krylov.KK_MIXED_BF16]


@pytest.fixture(scope="module", params=[56, 113, 140, 170, 250], ids=["fe56", "fe113", "fe140", "fe170", "fe250"])
def system(request):
    n = request.param
    sysd = make_system(n_atoms=n, seed=20_000 + n)
    return sysd, expansion_point(sysd)


@pytest.mark.parametrize("precision", PRECISIONS, ids=["fp64", "f16x3", "bf16"])
def test_ksplit_responses_and_kernel(system, precision):
    sysd, ep = system
    n = sysd["n_atoms"]
    h = handle_from_expansion(sysd, ep, precision)
    try:
        vs = np.random.default_rng(n).standard_normal((5, 2 * n))
        got = h.density_response_batch(t(vs)).cpu().numpy()
        errs = [rel(got[i], response(sysd, ep, vs[i])) for i in range(len(vs))]
        kd, info = h.krylov_kernel_apply(t(sysd["delta"]), 6)
        ek = rel(kd.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 6))
        print(f"{n} atoms (Nb {sysd['n_basis']}), precision {precision}: responses max {max(errs):.2e}, "
              f"kernel {ek:.2e}, rank {info.rank_used}", flush=True)
        assert max(errs) < TOL[precision], errs
        assert ek < TOL[precision], ek
    finally:
        h.close()


def test_ksplit_breakdown_fp64():
    """delta in a 2-dimensional invariant subspace of K0 J on the 56-atom cluster (four
    chunks): the expansion stops at rank 2 with KK_BREAKDOWN, every later kernel of the
    update returns at once, and the result is the oracle's (which stops there too)."""
    from oracle.krylov import jacobian_exact
    sysd = make_system(n_atoms=56, seed=20_056)
    ep = expansion_point(sysd)
    J = jacobian_exact(sysd, ep)
    lam, vec = np.linalg.eig(-J)
    real = np.argsort(np.abs(lam.imag))[:2]
    delta = np.real(vec[:, real[0]]) * 0.01 + np.real(vec[:, real[1]]) * 0.02
    h = handle_from_expansion(sysd, ep)
    try:
        x, info = h.krylov_kernel_apply(t(delta), 6)
        ref = kernel_apply(sysd, ep, delta, 6)
        err = rel(x.cpu().numpy(), ref)
        print(f"56 atoms breakdown: rank {info.rank_used}, status {info.status}, error {err:.2e}", flush=True)
        assert info.rank_used == 2 and info.status == krylov.KK_BREAKDOWN
        assert err < 1e-10
    finally:
        h.close()


@pytest.mark.parametrize("precision", PRECISIONS, ids=["fp64", "f16x3", "bf16"])
def test_ksplit_dense_preconditioner(system, precision):
    """A dense K0 (the fused step then leaves the preconditioning to its own launch after
    each response) at every size of the module, and for FP64 also the adaptive-rank call (a
    solve after each direction, checked against the oracle's stopping rank; the split forms'
    rounding could move a stopping rank across the tolerance), against the oracle."""
    sysd, ep = system
    n2 = 2 * sysd["n_atoms"]
    K0 = -np.eye(n2) + 0.05 * np.random.default_rng(13).standard_normal((n2, n2))
    h = handle_from_expansion(sysd, ep, precision)
    try:
        got, info = h.krylov_kernel_apply(t(sysd["delta"]), 5, K0=t(K0))
        e1 = rel(got.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 5, K0))
        print(f"{sysd['n_atoms']} atoms, precision {precision}: dense K0 {e1:.2e} (rank {info.rank_used})",
              flush=True)
        assert e1 < TOL[precision]
        if precision == krylov.KK_FP64:
            ga, ia = h.krylov_kernel_apply_adaptive(t(sysd["delta"]), 10, 0.1)
            ra, pa = kernel_apply(sysd, ep, sysd["delta"], 10, tol=0.1, return_parts=True)
            e2 = rel(ga.cpu().numpy(), ra)
            print(f"  adaptive {e2:.2e} (rank {ia.rank_used}, oracle {pa['rank']})", flush=True)
            assert ia.rank_used == pa["rank"] and e2 < TOL[precision]
    finally:
        h.close()
