"""Split-precision paths against the FP64 oracle: FP16 x 3 MFMA products, and
BF16 products with their refinement products (every test runs for both forms).

Bound: 1e-6 relative (2-norm) on every response and on the Krylov kernel
result, the accuracy the mixed-precision forms are held to; the measured
errors are ~1e-8..1e-7 and printed.
"""

import numpy as np
import pytest

from tests.gpu_helpers import handle_from_expansion, rel, t

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-6

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from oracle.response import response  # noqa: E402
from paper_2303_03529_amd.krylov import KK_MIXED_BF16, KK_MIXED_F16  # noqa: E402
from synth import make_system  # noqa: E402


def _case(n_cells=None, n_atoms=None, seed=0, precision=KK_MIXED_F16, **kw):
    sysd = make_system(n_cells, n_atoms=n_atoms, seed=seed, **kw)
    ep = expansion_point(sysd)
    return sysd, ep, handle_from_expansion(sysd, ep, precision)


@pytest.fixture(scope="module", params=[KK_MIXED_F16, KK_MIXED_BF16], ids=["f16x3", "bf16"])
def precision(request):
    return request.param


@pytest.fixture(scope="module")
def fe16m(precision):
    case = _case(2, seed=16, precision=precision)
    yield case
    case[2].close()


@pytest.fixture(scope="module")
def fe128m(precision):
    case = _case(4, seed=128, precision=precision)
    yield case
    case[2].close()


def test_mixed_response_fe16(fe16m):
    sysd, ep, h = fe16m
    V = np.random.default_rng(1).standard_normal((3, 2 * sysd["n_atoms"]))
    got = h.density_response_batch(t(V)).cpu().numpy()
    errs = [rel(got[b], response(sysd, ep, V[b])) for b in range(3)]
    print("mixed response errors fe16", errs)
    assert max(errs) < TOL_MIXED


def test_mixed_response_fe16_full_chunks(fe16m):
    """More directions than one launch takes (several full chunks and a partial one):
    every direction's operands are split in the chunk's single launch."""
    sysd, ep, h = fe16m
    V = np.random.default_rng(11).standard_normal((19, 2 * sysd["n_atoms"]))
    got = h.density_response_batch(t(V)).cpu().numpy()
    errs = [rel(got[b], response(sysd, ep, V[b])) for b in range(V.shape[0])]
    assert max(errs) < TOL_MIXED, errs


def test_mixed_response_fe128(fe128m):
    sysd, ep, h = fe128m
    V = np.random.default_rng(2).standard_normal((2, 2 * sysd["n_atoms"]))
    got = h.density_response_batch(t(V)).cpu().numpy()
    errs = [rel(got[b], response(sysd, ep, V[b])) for b in range(2)]
    print("mixed response errors fe128", errs)
    assert max(errs) < TOL_MIXED


def test_mixed_kernel_fe16(fe16m):
    sysd, ep, h = fe16m
    got, info = h.krylov_kernel_apply(t(sysd["delta"]), 4)
    err = rel(got.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 4))
    print("mixed kernel error fe16", err)
    assert info.rank_used == 4 and err < TOL_MIXED


def test_mixed_kernel_fe128(fe128m):
    sysd, ep, h = fe128m
    got, info = h.krylov_kernel_apply(t(sysd["delta"]), 8)
    err = rel(got.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 8))
    print("mixed kernel error fe128", err)
    assert info.rank_used == 8 and err < TOL_MIXED


@pytest.mark.parametrize("n_atoms", [1, 37, 129, 257])
def test_mixed_ragged_cluster(n_atoms, precision):
    """Ragged sizes: 1 atom (one tile, mostly padding), 37, 129 (padded 1280), 257 (Nb = 2313,
    above the small-shape limit: the large 256 x 128 products, padded 2560)."""
    sysd, ep, h = _case(n_atoms=n_atoms, seed=10_000 + n_atoms, precision=precision)
    try:
        v = np.random.default_rng(7).standard_normal(2 * n_atoms)
        got = h.density_response_batch(t(v)).cpu().numpy()[0]
        err = rel(got, response(sysd, ep, v))
        print(f"precision {precision}, {n_atoms} atoms: response error {err:.2e}")
        assert err < TOL_MIXED
    finally:
        h.close()


def test_mixed_is_deterministic(fe128m):
    sysd, ep, h = fe128m
    v = t(np.random.default_rng(3).standard_normal(2 * sysd["n_atoms"]))
    a = h.density_response_batch(v).cpu().numpy()
    b = h.density_response_batch(v).cpu().numpy()
    assert np.array_equal(a, b)
