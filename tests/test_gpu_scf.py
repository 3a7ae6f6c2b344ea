"""SCF acceleration and extended-Lagrangian electronic steps on the GPU,
against the oracle (Sec. III.C, II.F)."""

import numpy as np
import pytest

from tests.gpu_helpers import handle_from_expansion, rel, t

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from oracle.scf import net_q_of_n, scf as oracle_scf, xlbomd_update as oracle_xl  # noqa: E402
from paper_2303_03529_amd import scf as gpu_scf  # noqa: E402
from synth import make_system  # noqa: E402


@pytest.fixture(scope="module")
def fe16():
    sysd = make_system(2, seed=16)
    ep = expansion_point(sysd)
    return sysd, ep, handle_from_expansion(sysd, ep)


def test_ground_state_charges(fe16):
    sysd, ep, h = fe16
    got = h.ground_state_charges(t(sysd["valence"])).cpu().numpy()
    ref = net_q_of_n(sysd, sysd["n_ref"], ep["Z"])
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_adaptive_rank_kernel(fe16):
    sysd, ep, h = fe16
    for tol in (0.3, 0.05, 1e-3):
        got, info = h.krylov_kernel_apply_adaptive(t(sysd["delta"]), 12, tol)
        ref, parts = kernel_apply(sysd, ep, sysd["delta"], 12, return_parts=True, tol=tol)
        assert info.rank_used == parts["rank"], tol
        assert abs(info.ls_residual - parts["ls_residual"]) < 1e-10
        assert rel(got.cpu().numpy(), ref) < 1e-10


def test_xlbomd_update_kernel(fe16):
    sysd, ep, h = fe16
    rng = np.random.default_rng(3)
    n2 = 2 * sysd["n_atoms"]
    hist, Kf, c = rng.standard_normal((5, n2)), rng.standard_normal(n2), rng.standard_normal(5)
    got = h.xlbomd_update(t(hist), t(Kf), 1.7, 0.02, t(c)).cpu().numpy()
    assert np.abs(got - oracle_xl(hist, Kf, 1.7, 0.02, c)).max() < 1e-13 * np.abs(got).max()


def test_kernel_mixer_scf_matches_oracle():
    """Same fixed point, same iteration count (+-1), residual histories that agree early."""
    sysd = make_system(2, seed=16)
    kw = dict(tol=1e-10, max_iter=60, m_max=8, rank_tol=0.1, switch_at=10.0)
    n_gpu, h_gpu = gpu_scf.scf(sysd, sysd["n_ref"], **kw)
    n_ref, h_ref = oracle_scf(sysd, sysd["n_ref"], **kw)
    print("GPU SCF", [f"{x['rms']:.1e}/{x['rank']}" for x in h_gpu])
    print("oracle SCF", [f"{x['rms']:.1e}/{x['rank']}" for x in h_ref])
    assert h_gpu[-1]["mode"] == "done" and h_ref[-1]["mode"] == "done"
    assert abs(len(h_gpu) - len(h_ref)) <= 1
    for a, b in list(zip(h_gpu, h_ref))[:3]:
        assert abs(a["rms"] - b["rms"]) < 1e-8 * b["rms"] + 1e-13
    assert np.abs(n_gpu - n_ref).max() < 1e-8


def test_xlbomd_electrons_stay_near_ground_state():
    """From a converged n perturbed slightly, the extended-Lagrangian update keeps the residual small."""
    sysd = make_system(2, seed=16)
    n_star, _ = oracle_scf(sysd, sysd["n_ref"], tol=1e-11, max_iter=60, m_max=8, rank_tol=0.1, switch_at=10.0)
    start = n_star + 1e-3 * np.random.default_rng(5).standard_normal(n_star.size)
    res, n_end = gpu_scf.xlbomd_electrons(sysd, start, steps=12, kappa=1.0, m_max=6, rank_tol=0.05)
    print("XL-BOMD residuals", [f"{r:.1e}" for r in res])
    assert max(res) < 10 * res[0]


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-6)], ids=["fp64", "split"])
def test_kernel_mixer_scf_fe128_reaches_the_oracle_fixed_point(precision, tol):
    """128-atom bcc Fe: the GPU SCF with the adaptive-rank kernel mixer converges, and the
    density it returns is a fixed point of the oracle's own map q[n] (independent
    diagonalization and Mulliken sums on the CPU)."""
    from oracle.scf import rms
    sysd = make_system(4, seed=128)
    n_gpu, hist = gpu_scf.scf(sysd, sysd["n_ref"], tol=tol, max_iter=60, m_max=8, rank_tol=0.1, switch_at=10.0,
                              precision=precision)
    print("GPU SCF fe128", [f"{x['rms']:.1e}/{x['rank']}" for x in hist])
    assert hist[-1]["mode"] == "done"
    res = rms(net_q_of_n(sysd, n_gpu) - n_gpu)
    print(f"oracle residual at the GPU fixed point: {res:.2e}")
    assert res < 2 * tol
