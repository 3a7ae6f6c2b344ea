"""Batching form at its configured shape: the 64 open bcc-Fe clusters (atom
counts synth.cluster_sizes(64, 64), 22-248 atoms, Nb up to 2232), rank 6, in
one graph launch per batched update, FP64 and split precision, with each tile
class forced once (every system on the large tiles, then every system on the
64 x 64 tiles) and once autotuned.

The library is prepared from a device eigensolve (caller_setup), independent
of the oracle's eigenvectors; every system's K delta is compared, one by one,
with the oracle's stored value (tests/golden/clusters64_oracle.json, written
by make_oracle_golden.py, which calls only the oracle). Bounds: 1e-10 (FP64)
and 1e-6 (split) relative 2-norm per system.
"""

import json
import os

import numpy as np
import pytest

from tests.gpu_helpers import DEV, rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2303_03529_amd import krylov  # noqa: E402
from paper_2303_03529_amd.caller_setup import DeviceSystem  # noqa: E402
from synth import make_system  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "clusters64_oracle.json")
TOL = {krylov.KK_FP64: 1e-10, krylov.KK_MIXED_F16: 1e-6}
LARGE_ONLY, SMALL_ONLY = 0, 1 << 30   # tile-class thresholds on the padded size


@pytest.fixture(scope="module")
def golden():
    return json.load(open(GOLDEN))


@pytest.fixture(scope="module")
def clusters(golden):
    """(system dict, device expansion for kk_batch_prepare, delta) for each cluster."""
    out = []
    for s in golden["systems"]:
        sysd = make_system(n_atoms=s["n_atoms"], seed=s["seed"])
        e = DeviceSystem(sysd, DEV).expansion()
        dev = dict(offsets=sysd["offsets"], S=e["S"], Z=e["Z"], Q_up=e["Q_up"], Q_dn=e["Q_dn"],
                   eps_up=e["eps_up"], eps_dn=e["eps_dn"], gamma=e["gamma"], W=sysd["W"], kT=sysd["kT"],
                   n_electrons=sysd["n_electrons"])
        out.append((sysd, dev, t(sysd["delta"])))
    return out


def _errors(outs, golden):
    return [rel(o.cpu().numpy(), s["Kdelta"]) for o, s in zip(outs, golden["systems"])]


@pytest.mark.parametrize("precision", [krylov.KK_FP64, krylov.KK_MIXED_F16], ids=["fp64", "split_f16"])
def test_batch64_every_system_vs_oracle(clusters, golden, precision):
    m = golden["rank"]
    assert min(golden["sizes"]) < 30 and sum(n > 240 for n in golden["sizes"]) >= 2
    b = krylov.Batch().prepare([d for _, d, _ in clusters], precision)
    try:
        deltas = [d for _, _, d in clusters]
        # the autotuner first (it runs on the first update of a fresh batch), then each class forced
        for label, th in (("autotuned", None), ("large tiles", LARGE_ONLY), ("64x64 tiles", SMALL_ONLY)):
            if th is not None:
                b.set_tuning(th, 2)
                assert b.tuning()["small_np_max"] == th
            outs, infos = b.krylov_kernel_apply(deltas, m)
            # a second replay of the same graph with eager GPU work in between
            torch.cuda.synchronize()
            _ = (deltas[0] * 2.0).sum().item()
            outs2, _ = b.krylov_kernel_apply(deltas, m, outs=[torch.empty_like(o) for o in outs])
            errs = _errors(outs, golden)
            errs2 = _errors(outs2, golden)
            worst = int(np.argmax(errs))
            print(f"batch64 precision {precision}, {label} ({b.tuning()}): max rel err {max(errs):.2e} "
                  f"(system {worst}, {golden['sizes'][worst]} atoms), median {np.median(errs):.2e}; "
                  f"replay 2 max {max(errs2):.2e}", flush=True)
            assert all(i.rank_used == s["rank_used"] for i, s in zip(infos, golden["systems"]))
            assert max(errs) < TOL[precision], (label, worst, max(errs))
            assert max(errs2) < TOL[precision], (label, max(errs2))
    finally:
        b.close()


def test_batch64_set_tuning_validates():
    sysd = make_system(n_atoms=16, seed=10_000)
    e = DeviceSystem(sysd, DEV).expansion()
    b = krylov.Batch().prepare([dict(offsets=sysd["offsets"], S=e["S"], Z=e["Z"], Q_up=e["Q_up"],
                                     Q_dn=e["Q_dn"], eps_up=e["eps_up"], eps_dn=e["eps_dn"], gamma=e["gamma"],
                                     W=sysd["W"], kT=sysd["kT"], n_electrons=sysd["n_electrons"])])
    try:
        for bad in ((-1, 2), (0, 0), (0, 9)):
            with pytest.raises(krylov.KKError):
                b.set_tuning(*bad)
        b.set_tuning(0, 4)
        assert b.tuning() == dict(small_np_max=0, workgroups_per_cu=4, update_ms=0.0)
    finally:
        b.close()
