"""The HIP path at the benchmark's full size (1024-atom bcc Fe, Nb = 9216,
m = 12), in the launch configuration bench.py times.

The library is prepared from the device eigensolve (caller_setup), the same
inputs bench.py uses, so it is independent of the oracle's eigenvectors; only
basis-invariant outputs are compared with the oracle's stored values
(tests/golden/fe1024_oracle.json, written by make_oracle_golden.py, which
calls only the oracle). Properties that hold at any size are checked too.
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fe1024_oracle.json")
TOL_FP64 = 1e-10
TOL_MIXED = 1e-6


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file not generated")
    return json.load(open(GOLDEN))


@pytest.fixture(scope="module")
def fe1024():
    sysd = make_system(8, seed=1024)
    return sysd


@pytest.fixture(scope="module")
def h64(fe1024):
    h = handle_from_device_setup(fe1024, KK_FP64)
    yield h
    h.close()


def test_fullsize_mu(h64, golden):
    assert abs(h64.mu - golden["mu"]) < 1e-11 * abs(golden["mu"])


def test_fullsize_response_vs_oracle(fe1024, h64, golden):
    v = krylov_vectors(fe1024["n_atoms"], 1, golden["v_seed"])[0]
    got = h64.density_response_batch(t(v)).cpu().numpy()[0]
    err = rel(got, golden["q1"])
    print(f"1024-atom response vs oracle: {err:.2e}")
    assert err < TOL_FP64


def test_fullsize_kernel_vs_oracle(fe1024, h64, golden):
    got, info = h64.krylov_kernel_apply(t(fe1024["delta"]), golden["rank"])
    assert info.rank_used == golden["rank_used"]
    err = rel(got.cpu().numpy(), golden["Kdelta"])
    print(f"1024-atom rank-12 kernel vs oracle: {err:.2e}")
    assert err < TOL_FP64


def test_fullsize_invariants(fe1024, h64):
    """Charge conservation, response symmetry and linearity at full size."""
    N = fe1024["n_atoms"]
    rng = np.random.default_rng(99)
    a, b = rng.standard_normal((2, 2 * N))
    q = h64.density_response_batch(t(np.stack([a, b, 2 * a - 3 * b]))).cpu().numpy()
    assert abs(q[0][:N].sum()) < 1e-12 * np.abs(q[0]).sum()

    def gam(x):
        return np.concatenate([fe1024["gamma"] @ x[:N], fe1024["W"] * x[N:]])

    lhs, rhs = gam(a) @ q[1], gam(b) @ q[0]
    assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), abs(rhs))
    assert rel(q[2], 2 * q[0] - 3 * q[1]) < 1e-12


@pytest.mark.parametrize("precision", [KK_MIXED_F16, KK_MIXED_BF16], ids=["f16x3", "bf16"])
def test_fullsize_mixed_vs_oracle(fe1024, golden, precision):
    h = handle_from_device_setup(fe1024, precision)
    try:
        v = krylov_vectors(fe1024["n_atoms"], 1, golden["v_seed"])[0]
        q = h.density_response_batch(t(v)).cpu().numpy()[0]
        got, info = h.krylov_kernel_apply(t(fe1024["delta"]), golden["rank"])
        e_q = rel(q, golden["q1"])
        e_k = rel(got.cpu().numpy(), golden["Kdelta"])
        print(f"1024-atom split-precision ({precision}) errors: response {e_q:.2e}, kernel {e_k:.2e}")
        assert e_q < TOL_MIXED and e_k < TOL_MIXED
    finally:
        h.close()
