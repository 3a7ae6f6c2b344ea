"""Batched form: uneven clusters in one graph launch, against the oracle and
against the single-system path."""

import numpy as np
import pytest

from tests.gpu_helpers import rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from paper_2303_03529_amd import krylov  # noqa: E402
from synth import make_system  # noqa: E402

SIZES = [16, 23, 40, 17, 61, 33]


def _systems():
    out = []
    for i, n in enumerate(SIZES):
        sysd = make_system(n_atoms=n, seed=10_000 + i)
        ep = expansion_point(sysd)
        dev = dict(offsets=sysd["offsets"], S=t(sysd["S"]), Z=t(ep["Z"]), Q_up=t(ep["Q"][0]), Q_dn=t(ep["Q"][1]),
                   eps_up=t(ep["eps"][0]), eps_dn=t(ep["eps"][1]), gamma=t(sysd["gamma"]), W=sysd["W"],
                   kT=sysd["kT"], n_electrons=sysd["n_electrons"])
        out.append((sysd, ep, dev))
    return out


@pytest.fixture(scope="module")
def systems():
    return _systems()


@pytest.mark.parametrize("precision,tol", [(krylov.KK_FP64, 1e-10), (krylov.KK_MIXED_F16, 1e-6)])
def test_batch_matches_oracle(systems, precision, tol):
    b = krylov.Batch().prepare([d for _, _, d in systems], precision)
    m = 6
    refs = [kernel_apply(s, ep, s["delta"], m) for s, ep, _ in systems]
    # three replays of the captured graph with different inputs, eager work in between
    for rep, scale in enumerate((1.0, -2.0, 0.5)):
        deltas = [t(scale * s["delta"]) for s, _, _ in systems]
        outs, infos = b.krylov_kernel_apply(deltas, m)
        errs = [rel(o.cpu().numpy(), scale * r) for o, r in zip(outs, refs)]
        print(f"batch precision {precision} replay {rep}: max rel err {max(errs):.2e}")
        assert max(errs) < tol
        assert all(i.rank_used == m for i in infos)
        h = krylov.Handle()  # eager single-system work between replays
        s0, ep0, d0 = systems[0]
        h.prepare(d0["offsets"], d0["S"], d0["Z"], d0["Q_up"], d0["Q_dn"], d0["eps_up"], d0["eps_dn"],
                  d0["gamma"], d0["W"], d0["kT"], d0["n_electrons"], precision)
        single, _ = h.krylov_kernel_apply(t(scale * s0["delta"]), m)
        assert rel(single.cpu().numpy(), outs[0].cpu().numpy()) < tol
        h.close()
        torch.cuda.synchronize()
    tune = b.tuning()
    print("batch tuning", tune)
    assert tune["workgroups_per_cu"] in (1, 2, 4)
    b.close()


def test_batch_breakdown_is_per_system(systems):
    """A zero residual in one system stops only that system's expansion."""
    b = krylov.Batch().prepare([d for _, _, d in systems], krylov.KK_FP64)
    deltas = [t(s["delta"]) for s, _, _ in systems]
    deltas[2] = torch.zeros_like(deltas[2])
    outs, infos = b.krylov_kernel_apply(deltas, 4)
    assert infos[2].rank_used == 0 and not torch.any(outs[2])
    s, ep, _ = systems[1]
    assert infos[1].rank_used == 4
    assert rel(outs[1].cpu().numpy(), kernel_apply(s, ep, s["delta"], 4)) < 1e-10
    b.close()
