"""The allocation-free entry point krylov_kernel_apply_noalloc, called through
the C ABI, against krylov_kernel_apply on the same handles: two calls in a
row (a 128-atom bcc cell, then a smaller 37-atom open cluster, so the second
call reuses the fixed scratch array holding the first call's data), in FP64
and in the split-precision forms, plus the FP64 results against the oracle, the
split forms' stream-K products in the scratch array, FP64 handles on the large tile
class of small systems, and the refusal of a handle whose workspace does not fit."""

import numpy as np
import pytest

from tests.gpu_helpers import handle_from_expansion, rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from paper_2303_03529_amd import krylov  # noqa: E402
from synth import make_system  # noqa: E402

TOL = {krylov.KK_FP64: 1e-10, krylov.KK_MIXED_F16: 1e-6, krylov.KK_MIXED_BF16: 1e-6}


@pytest.fixture(scope="module")
def systems():
    out = []
    for sysd in (make_system(4, seed=128), make_system(n_atoms=37, seed=10_037)):
        out.append((sysd, expansion_point(sysd)))
    return out


@pytest.mark.parametrize("precision", [krylov.KK_FP64, krylov.KK_MIXED_F16, krylov.KK_MIXED_BF16],
                         ids=["fp64", "split_f16", "bf16"])
def test_noalloc_matches_apply_on_two_calls(systems, precision):
    m = 8
    for call, (sysd, ep) in enumerate(systems):
        print(f"no-alloc call {call}: {sysd['n_atoms']} atoms, precision {precision}", flush=True)
        h = handle_from_expansion(sysd, ep, precision)
        try:
            d = t(sysd["delta"])
            ref, info_ref = h.krylov_kernel_apply(d, m)
            out = torch.full_like(d, float("nan"))
            got, info = h.krylov_kernel_apply_noalloc(d, m, out=out)
            torch.cuda.synchronize()
            assert got.data_ptr() == out.data_ptr()
            err = rel(got.cpu().numpy(), ref.cpu().numpy())
            print(f"  vs krylov_kernel_apply: {err:.2e}; rank {info.rank_used}", flush=True)
            assert info.rank_used == info_ref.rank_used == m
            assert err < TOL[precision]
            if precision == krylov.KK_FP64:
                e_or = rel(got.cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], m))
                print(f"  vs oracle: {e_or:.2e}", flush=True)
                assert e_or < TOL[precision]
            # the entry point after a graph replay and before one: both keep agreeing
            again, _ = h.krylov_kernel_apply(d, m)
            assert rel(again.cpu().numpy(), ref.cpu().numpy()) < 1e-15
        finally:
            h.close()


@pytest.mark.parametrize("precision", [krylov.KK_MIXED_F16, krylov.KK_MIXED_BF16], ids=["split_f16", "bf16"])
def test_noalloc_stream_k_products(precision):
    """The split forms' stream-K products (170-atom cluster, Nb = 1530: two partial slots per
    item in the scratch array, BF16 91 MiB of it), then a 128-atom cell in the same array:
    each against krylov_kernel_apply on the same handle."""
    cases = [make_system(n_atoms=170, seed=20_170), make_system(4, seed=128)]
    for call, sysd in enumerate(cases):
        ep = expansion_point(sysd)
        print(f"no-alloc stream-K call {call}: {sysd['n_atoms']} atoms, precision {precision}", flush=True)
        h = handle_from_expansion(sysd, ep, precision)
        try:
            d = t(sysd["delta"])
            ref, _ = h.krylov_kernel_apply(d, 6)
            got, info = h.krylov_kernel_apply_noalloc(d, 6, out=torch.full_like(d, float("nan")))
            torch.cuda.synchronize()
            err = rel(got.cpu().numpy(), ref.cpu().numpy())
            print(f"  vs krylov_kernel_apply: {err:.2e}; rank {info.rank_used}", flush=True)
            assert info.rank_used == 6 and err < 1e-15
        finally:
            h.close()


def test_noalloc_fp64_large_tile_class():
    """FP64 handles on the 128 x 128 tiles below a padded size of 2304 (250 atoms: full-tile
    forward in three rounds of workgroups, 85 MB of the scratch array; then 140 atoms, one
    round) through the allocation-free entry point, each against krylov_kernel_apply on the
    same handle, bit for bit."""
    cases = [make_system(n_atoms=250, seed=20_250), make_system(n_atoms=140, seed=20_140)]
    for call, sysd in enumerate(cases):
        ep = expansion_point(sysd)
        print(f"no-alloc FP64 call {call}: {sysd['n_atoms']} atoms", flush=True)
        h = handle_from_expansion(sysd, ep, krylov.KK_FP64)
        try:
            d = t(sysd["delta"])
            ref, _ = h.krylov_kernel_apply(d, 6)
            got, info = h.krylov_kernel_apply_noalloc(d, 6, out=torch.full_like(d, float("nan")))
            torch.cuda.synchronize()
            err = rel(got.cpu().numpy(), ref.cpu().numpy())
            print(f"  vs krylov_kernel_apply: {err:.2e}; rank {info.rank_used}", flush=True)
            assert info.rank_used == 6 and err == 0.0
        finally:
            h.close()


def test_noalloc_refuses_a_handle_that_does_not_fit():
    sysd = make_system(n_atoms=290, seed=10_290)   # Nb = 2610, padded 2688: 116 MB of Y
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, krylov.KK_FP64)
    try:
        d = t(sysd["delta"])
        out = torch.zeros_like(d)
        with pytest.raises(krylov.KKError) as e:
            h.krylov_kernel_apply_noalloc(d, 4, out=out)
        assert e.value.status == krylov.KK_EINVAL and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert not torch.any(out)  # nothing was enqueued
    finally:
        h.close()
