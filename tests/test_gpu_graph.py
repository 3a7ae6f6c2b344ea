"""The captured single-system update (a graph launch per call) against the
launch-by-launch path: the same handle with kernel timing on, which takes the
launch-by-launch path, and off, which replays the graph. Covered: several
replays with other GPU work between them, new inputs in the same and in new
buffers, input and output pointers that change between back-to-back replays, a
change of rank and of tolerance, a reverse pass that reuses the
forward's expansion, and a second prepare of the same handle."""

import numpy as np
import pytest

from tests.gpu_helpers import DEV, handle_from_expansion, rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from paper_2303_03529_amd import krylov  # noqa: E402
from synth import make_system  # noqa: E402

TOL = {krylov.KK_FP64: 1e-10, krylov.KK_MIXED_F16: 1e-6, krylov.KK_MIXED_BF16: 1e-6}
SAME = 1e-13  # both paths run the same kernels on the same inputs


def launch_by_launch(h, delta, m, tol=None):
    h.profile_enable(True)
    try:
        if tol is None:
            out, info = h.krylov_kernel_apply(delta, m)
        else:
            out, info = h.krylov_kernel_apply_adaptive(delta, m, tol)
    finally:
        h.profile_enable(False)
    return out.clone(), info


def close(a, b):
    a = a.cpu().numpy()
    b = b.cpu().numpy()
    return float(np.linalg.norm(a - b)) <= SAME * float(np.linalg.norm(b))


@pytest.mark.parametrize("precision", [krylov.KK_FP64, krylov.KK_MIXED_F16, krylov.KK_MIXED_BF16],
                         ids=["fp64", "split", "bf16"])
def test_graph_replays_match_launch_by_launch(precision):
    sysd = make_system(2, seed=16)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, precision)
    try:
        n2 = 2 * h.n_atoms
        rng = np.random.default_rng(2303)
        deltas = [sysd["delta"]] + [1e-2 * rng.standard_normal(n2) for _ in range(3)]
        buf = t(deltas[0])
        out = torch.empty_like(buf)
        for i, d in enumerate(deltas):
            buf.copy_(t(d))  # same buffer, new contents
            ref, ref_info = launch_by_launch(h, buf, 6)
            g, info = h.krylov_kernel_apply(buf, 6, out=out)
            assert close(g, ref), i
            assert info.rank_used == ref_info.rank_used
            noise = torch.randn(4096, 64, device=DEV, dtype=torch.float64) @ torch.randn(64, 64, device=DEV,
                                                                                          dtype=torch.float64)
            g2, _ = h.krylov_kernel_apply(t(d), 6)  # new buffers
            assert close(g2, ref), i
            del noise
            if i == 0:
                assert rel(g.cpu().numpy(), kernel_apply(sysd, ep, d, 6)) < TOL[precision]
        g3, _ = h.krylov_kernel_apply(buf, 4)  # another rank: a new capture
        assert close(g3, launch_by_launch(h, buf, 4)[0])
        ga, ia = h.krylov_kernel_apply_adaptive(buf, 8, 1e-6)
        ra, ria = launch_by_launch(h, buf, 8, 1e-6)
        assert close(ga, ra) and ia.rank_used == ria.rank_used
        ga2, _ = h.krylov_kernel_apply_adaptive(buf, 8, 1e-3)  # another tolerance
        assert close(ga2, launch_by_launch(h, buf, 8, 1e-3)[0])
    finally:
        h.close()


def test_graph_with_reverse_pass_and_second_prepare():
    sysd = make_system(2, seed=16)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, krylov.KK_FP64)
    try:
        delta = t(sysd["delta"])
        kd, _ = h.krylov_kernel_apply(delta, 6)
        xbar = t(np.linspace(-1.0, 1.0, 2 * h.n_atoms))
        reuse = h.krylov_kernel_adjoint(delta, 6, xbar, reuse_forward=True, want_H=False)
        fresh = h.krylov_kernel_adjoint(delta, 6, xbar, reuse_forward=False, want_H=False)
        assert close(reuse["delta"], fresh["delta"])
        kd2, _ = h.krylov_kernel_apply(delta, 6)  # after the reverse pass's allocations
        assert close(kd2, kd)
        other = make_system(2, seed=17)
        ep2 = expansion_point(other)
        h.prepare(other["offsets"], t(other["S"]), t(ep2["Z"]), t(ep2["Q"][0]), t(ep2["Q"][1]),
                  t(ep2["eps"][0]), t(ep2["eps"][1]), t(other["gamma"]), other["W"], other["kT"],
                  other["n_electrons"], krylov.KK_FP64)
        kd3, _ = h.krylov_kernel_apply(t(other["delta"]), 6)
        assert rel(kd3.cpu().numpy(), kernel_apply(other, ep2, other["delta"], 6)) < TOL[krylov.KK_FP64]
    finally:
        h.close()


def test_graph_recapture_without_host_sync():
    """Calls that change the rank (a new capture) or re-prepare the handle, issued back to back
    with no host synchronization in between, while the previous replay is still running (a
    128-atom update takes milliseconds): every result must equal the launch-by-launch one.
    A re-prepare of the same shape with the same W and kT keeps the graph; another W recaptures."""
    sysd = make_system(4, seed=128)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, krylov.KK_FP64)
    try:
        delta = t(sysd["delta"])
        args = (sysd["offsets"], t(sysd["S"]), t(ep["Z"]), t(ep["Q"][0]), t(ep["Q"][1]), t(ep["eps"][0]),
                t(ep["eps"][1]), t(sysd["gamma"]))
        plan = [(8, 1.0), (6, 1.0), (8, 1.0), (5, 1.0), (8, 1.05), (8, 1.05), (6, 1.0)]
        outs = []
        for m, wscale in plan:
            if wscale != 1.0 or (outs and plan[len(outs) - 1][1] != wscale):
                h.prepare(*args, sysd["W"] * wscale, sysd["kT"], sysd["n_electrons"], krylov.KK_FP64)
            o = torch.empty_like(delta)
            h.krylov_kernel_apply(delta, m, out=o, info=False)   # returns with the replay in flight
            outs.append(o)
        torch.cuda.synchronize()
        for (m, wscale), o in zip(plan, outs):
            h.prepare(*args, sysd["W"] * wscale, sysd["kT"], sysd["n_electrons"], krylov.KK_FP64)
            ref, _ = launch_by_launch(h, delta, m)
            assert close(o, ref), (m, wscale)
    finally:
        h.close()


@pytest.mark.parametrize("precision", [krylov.KK_FP64, krylov.KK_MIXED_F16], ids=["fp64", "split"])
def test_graph_pointer_changes_back_to_back(precision):
    """Replays of one captured update (same key) whose input and output pointers change
    from call to call (input only, output only, both, neither), issued back to back with no
    host synchronization: the graph reads each call's delta and writes each call's K delta
    where they are, and every output buffer ends up holding the launch-by-launch result of
    the last call that wrote it."""
    sysd = make_system(4, seed=128)
    ep = expansion_point(sysd)
    h = handle_from_expansion(sysd, ep, precision)
    try:
        n2 = 2 * h.n_atoms
        rng = np.random.default_rng(55)
        ins = [t(sysd["delta"])] + [t(1e-2 * rng.standard_normal(n2)) for _ in range(2)]
        outs = [torch.empty_like(ins[0]) for _ in range(4)]
        plan = [(0, 0), (0, 0), (1, 0), (1, 1), (2, 2), (0, 3), (2, 1), (2, 1)]
        last = {}
        for i, o in plan:
            h.krylov_kernel_apply(ins[i], 8, out=outs[o], info=False)
            last[o] = i
        torch.cuda.synchronize()
        got = {o: outs[o].clone() for o in last}
        for o, i in last.items():
            ref, _ = launch_by_launch(h, ins[i], 8)
            assert close(got[o], ref), (o, i)
        assert rel(got[3].cpu().numpy(), kernel_apply(sysd, ep, sysd["delta"], 8)) < TOL[precision]
    finally:
        h.close()
