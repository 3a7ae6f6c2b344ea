"""Precision form at 432 atoms (6x6x6 bcc Fe, Nb = 3888, rank 8): the FP64, the
split FP16 x 3 and the BF16 (with its refinement products) transforms against the
FP64 oracle, error per output.

Both handles are prepared from the device eigensolve (independent of the
oracle's eigenvectors); the oracle's basis-invariant results come from
tests/golden/fe432_oracle.json (make_oracle_golden.py, oracle only). Outputs
compared one by one: mu, the charge and magnetization halves of each of the
eight fixed-direction responses, and the rank-8 kernel result.
"""

import json
import os

import numpy as np
import pytest

from tests.gpu_helpers import handle_from_device_setup, rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2303_03529_amd.krylov import KK_FP64, KK_MIXED_BF16, KK_MIXED_F16  # noqa: E402
from synth import make_system, krylov_vectors  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fe432_oracle.json")
TOL = {KK_FP64: 1e-10, KK_MIXED_F16: 1e-6, KK_MIXED_BF16: 1e-6}
NAME = {KK_FP64: "fp64", KK_MIXED_F16: "split f16 x 3", KK_MIXED_BF16: "bf16 + refinement"}


@pytest.fixture(scope="module")
def golden():
    return json.load(open(GOLDEN))


@pytest.fixture(scope="module")
def fe432(golden):
    return make_system(golden["cells"], seed=golden["seed"])


@pytest.mark.parametrize("precision", [KK_FP64, KK_MIXED_F16, KK_MIXED_BF16], ids=["fp64", "split_f16", "bf16"])
def test_precision_form_per_output(fe432, golden, precision):
    N = fe432["n_atoms"]
    h = handle_from_device_setup(fe432, precision)
    try:
        vs = krylov_vectors(N, len(golden["q1"]), golden["v_seed"])
        q = h.density_response_batch(t(vs)).cpu().numpy()
        kd, info = h.krylov_kernel_apply(t(fe432["delta"]), golden["rank"])
        errs = {"mu": abs(h.mu - golden["mu"]) / abs(golden["mu"])}
        for i, ref in enumerate(golden["q1"]):
            ref = np.asarray(ref)
            errs[f"dq[{i}]"] = rel(q[i][:N], ref[:N])
            errs[f"dm[{i}]"] = rel(q[i][N:], ref[N:])
        errs["Kdelta"] = rel(kd.cpu().numpy(), golden["Kdelta"])
        print(f"432-atom errors vs FP64 oracle ({NAME[precision]}):")
        for k, v in errs.items():
            print(f"  {k:8s} {v:.2e}")
        assert info.rank_used == golden["rank_used"]
        assert errs["mu"] < 1e-12
        assert max(errs.values()) < TOL[precision]
    finally:
        h.close()
