"""Thin Python binding of libkrylov_kernel.so (C ABI in include/krylov_kernel.h).

Argument marshalling only: every step of the computation runs in the HIP
library. Tensors must be float64, contiguous, on a ROCm device; the handle's
stream is the current torch stream at creation unless one is given.
If the library is missing this module raises at import time instead of
falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libkrylov_kernel.so")

KK_OK, KK_BREAKDOWN = 0, 1
KK_EINVAL, KK_ENOMEM, KK_EHIP, KK_ENOTPREPARED, KK_ESINGULAR = -1, -2, -3, -4, -5
KK_FP64, KK_MIXED_F16, KK_MIXED_BF16 = 0, 1, 2
STATUS_NAMES = {0: "KK_OK", 1: "KK_BREAKDOWN", -1: "KK_EINVAL", -2: "KK_ENOMEM", -3: "KK_EHIP",
                -4: "KK_ENOTPREPARED", -5: "KK_ESINGULAR"}

# Every function the header declares, with (restype, argtypes).
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
SIGNATURES = {
    "kk_create": (_I, [ctypes.POINTER(_P), _P]),
    "kk_destroy": (_I, [_P]),
    "kk_prepare": (_I, [_P, _I, _P, _I, _P, _P, _P, _P, _P, _P, _P, _D, _D, _D, _I]),
    "kk_get_mu": (_I, [_P, ctypes.POINTER(_D)]),
    "density_response_batch": (_I, [_P, _I, _P, _P]),
    "mulliken_project": (_I, [_P, _I, _P, _P, _P]),
    "krylov_kernel_apply": (_I, [_P, _P, _I, _P, _P, _P]),
    "krylov_kernel_apply_adaptive": (_I, [_P, _P, _I, _D, _P, _P, _P]),
    "krylov_kernel_apply_noalloc": (_I, [_P, _P, _I, _P, _P, _P]),
    "kk_ground_state_charges": (_I, [_P, _P, _P]),
    "kk_xlbomd_update": (_I, [_P, _P, _I, _P, _D, _D, _P, _P]),
    "krylov_kernel_adjoint": (_I, [_P, _P, _I, _P, _P, _I, _P, _P, _P, _P, _P, _P, _P]),
    "kk_last_error": (ctypes.c_char_p, []),
    "kk_batch_create": (_I, [ctypes.POINTER(_P), _P]),
    "kk_batch_destroy": (_I, [_P]),
    "kk_batch_prepare": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I]),
    "krylov_kernel_apply_batch": (_I, [_P, _P, _I, _P, _P]),
    "kk_batch_tuning": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_D)]),
    "kk_batch_set_tuning": (_I, [_P, _I, _I]),
    "kk_profile_enable": (_I, [_P, _I]),
    "kk_profile_reset": (_I, [_P]),
    "kk_profile_read": (_I, [_P, _I, ctypes.POINTER(_D), ctypes.POINTER(_I)]),
}


class KKInfo(ctypes.Structure):
    _fields_ = [("rank_used", _I), ("status", _I), ("min_pivot", _D), ("max_pivot", _D),
                ("ls_residual", _D)]


class KKError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = load_library()


def last_error() -> str:
    return LIB.kk_last_error().decode()


def _check(status: int, where: str, ok=(KK_OK,)) -> int:
    if status not in ok:
        raise KKError(status, where, last_error())
    return status


def _dev(t, name: str, numel: int | None = None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor on the GPU")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class KrylovInfo:
    rank_used: int
    status: int
    min_pivot: float
    max_pivot: float
    ls_residual: float


class Handle:
    """One library handle bound to one HIP stream."""

    def __init__(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._h = ctypes.c_void_p()
        _check(LIB.kk_create(ctypes.byref(self._h), ctypes.c_void_p(stream.cuda_stream)), "kk_create")
        self.n_atoms = None
        self.n_basis = None

    def close(self):
        if self._h:
            _check(LIB.kk_destroy(self._h), "kk_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, offsets, S, Z, Q_up, Q_dn, eps_up, eps_dn, gamma, W: float, kT: float,
                n_electrons: float, precision: int = KK_FP64):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
        n, nb = len(off) - 1, int(off[-1])
        _check(LIB.kk_prepare(
            self._h, n, off.ctypes.data_as(ctypes.c_void_p), nb,
            _dev(S, "S", nb * nb), _dev(Z, "Z", nb * nb), _dev(Q_up, "Q_up", nb * nb),
            _dev(Q_dn, "Q_dn", nb * nb), _dev(eps_up, "eps_up", nb), _dev(eps_dn, "eps_dn", nb),
            _dev(gamma, "gamma", n * n), float(W), float(kT), float(n_electrons), int(precision)),
            "kk_prepare")
        self.n_atoms, self.n_basis = n, nb
        return self

    @property
    def mu(self) -> float:
        out = ctypes.c_double()
        _check(LIB.kk_get_mu(self._h, ctypes.byref(out)), "kk_get_mu")
        return out.value

    def density_response_batch(self, v, out=None):
        import torch
        v2 = v.reshape(-1, 2 * self.n_atoms)
        if out is None:
            out = torch.empty_like(v2)
        _check(LIB.density_response_batch(self._h, v2.shape[0], _dev(v2, "v"),
                                          _dev(out, "q1", v2.numel())), "density_response_batch")
        return out

    def mulliken_project(self, dD_up, dD_dn, out=None):
        import torch
        nb = self.n_basis
        batch = dD_up.numel() // (nb * nb)
        if out is None:
            out = torch.empty(batch, 2 * self.n_atoms, dtype=torch.float64, device=dD_up.device)
        _check(LIB.mulliken_project(self._h, batch, _dev(dD_up, "dD_up", batch * nb * nb),
                                    _dev(dD_dn, "dD_dn", batch * nb * nb),
                                    _dev(out, "dqm", batch * 2 * self.n_atoms)), "mulliken_project")
        return out

    def krylov_kernel_apply(self, delta, m: int, K0=None, out=None, info: bool = True):
        """K delta; returns (out, KrylovInfo or None). info=True synchronizes."""
        return self._apply("krylov_kernel_apply", delta, m, K0, out, info)

    def krylov_kernel_apply_noalloc(self, delta, m: int, K0=None, out=None, info: bool = True):
        """K delta through the entry point that allocates nothing (out must be given
        to avoid allocating it here); returns (out, KrylovInfo or None)."""
        return self._apply("krylov_kernel_apply_noalloc", delta, m, K0, out, info)

    def _apply(self, name, delta, m, K0, out, info):
        import torch
        n2 = 2 * self.n_atoms
        if out is None:
            out = torch.empty(n2, dtype=torch.float64, device=delta.device)
        k0p = _dev(K0, "K0", n2 * n2) if K0 is not None else ctypes.c_void_p()
        fn = getattr(LIB, name)
        if info:
            inf = KKInfo()
            _check(fn(self._h, _dev(delta, "delta", n2), int(m), k0p, _dev(out, "Kdelta", n2), ctypes.byref(inf)),
                   name, ok=(KK_OK, KK_BREAKDOWN, KK_ESINGULAR))
            return out, KrylovInfo(inf.rank_used, inf.status, inf.min_pivot, inf.max_pivot, inf.ls_residual)
        _check(fn(self._h, _dev(delta, "delta", n2), int(m), k0p, _dev(out, "Kdelta", n2), None), name)
        return out, None

    def krylov_kernel_apply_adaptive(self, delta, m_max: int, tol: float, K0=None, out=None):
        """Adaptive-rank K delta; returns (out, KrylovInfo). Synchronizes."""
        import torch
        n2 = 2 * self.n_atoms
        if out is None:
            out = torch.empty(n2, dtype=torch.float64, device=delta.device)
        k0p = _dev(K0, "K0", n2 * n2) if K0 is not None else ctypes.c_void_p()
        inf = KKInfo()
        _check(LIB.krylov_kernel_apply_adaptive(self._h, _dev(delta, "delta", n2), int(m_max), float(tol), k0p,
                                                _dev(out, "Kdelta", n2), ctypes.byref(inf)),
               "krylov_kernel_apply_adaptive", ok=(KK_OK, KK_BREAKDOWN, KK_ESINGULAR))
        return out, KrylovInfo(inf.rank_used, inf.status, inf.min_pivot, inf.max_pivot, inf.ls_residual)

    def krylov_kernel_adjoint(self, delta, m: int, Kdelta_bar, K0=None, reuse_forward: bool = False,
                              want_Kdelta: bool = False, want_H: bool = True):
        """Reverse pass of K delta for x_bar = Kdelta_bar. Synchronizes.

        Returns dict(delta, gamma, W, H_up, H_dn, Kdelta (or None), info): the
        gradients of the caller's L with respect to delta, gamma (through the
        response potentials), W (likewise, a 0-d tensor) and, with want_H, the
        expansion-point spin Hamiltonians (n_basis x n_basis each; else None).
        """
        import torch
        n, nb = self.n_atoms, self.n_basis
        n2 = 2 * n
        dev = delta.device
        kw = dict(dtype=torch.float64, device=dev)
        out = dict(delta=torch.empty(n2, **kw), gamma=torch.empty(n, n, **kw), W=torch.empty((), **kw),
                   H_up=torch.empty(nb, nb, **kw) if want_H else None,
                   H_dn=torch.empty(nb, nb, **kw) if want_H else None,
                   Kdelta=torch.empty(n2, **kw) if want_Kdelta and not reuse_forward else None)
        hup = _dev(out["H_up"], "H_bar_up", nb * nb) if want_H else ctypes.c_void_p()
        hdn = _dev(out["H_dn"], "H_bar_dn", nb * nb) if want_H else ctypes.c_void_p()
        k0p = _dev(K0, "K0", n2 * n2) if K0 is not None else ctypes.c_void_p()
        kdp = _dev(out["Kdelta"], "Kdelta", n2) if out["Kdelta"] is not None else ctypes.c_void_p()
        inf = KKInfo()
        _check(LIB.krylov_kernel_adjoint(
            self._h, _dev(delta, "delta", n2), int(m), k0p, _dev(Kdelta_bar, "Kdelta_bar", n2),
            1 if reuse_forward else 0, kdp, _dev(out["delta"], "delta_bar", n2),
            _dev(out["gamma"], "gamma_bar", n * n), _dev(out["W"], "W_bar", 1),
            hup, hdn, ctypes.byref(inf)),
            "krylov_kernel_adjoint", ok=(KK_OK, KK_BREAKDOWN))
        out["info"] = KrylovInfo(inf.rank_used, inf.status, inf.min_pivot, inf.max_pivot, inf.ls_residual)
        return out

    def ground_state_charges(self, reference=None, out=None):
        """q[n] at the prepared point; reference (device, N) = neutral-atom populations."""
        import torch
        if out is None:
            out = torch.empty(2 * self.n_atoms, dtype=torch.float64, device="cuda")
        ref = _dev(reference, "reference", self.n_atoms) if reference is not None else ctypes.c_void_p()
        _check(LIB.kk_ground_state_charges(self._h, ref, _dev(out, "qm", 2 * self.n_atoms)),
               "kk_ground_state_charges")
        return out

    def xlbomd_update(self, n_hist, Kf, kappa: float, alpha: float, c, out=None):
        """n_hist (k_max+1, 2N) with row k = n(t - k dt); c (k_max+1,) on the device."""
        import torch
        n2 = 2 * self.n_atoms
        kmax = n_hist.shape[0] - 1
        if out is None:
            out = torch.empty(n2, dtype=torch.float64, device=n_hist.device)
        _check(LIB.kk_xlbomd_update(self._h, _dev(n_hist, "n_hist", (kmax + 1) * n2), kmax, _dev(Kf, "Kf", n2),
                                    float(kappa), float(alpha), _dev(c, "c", kmax + 1), _dev(out, "n_new", n2)),
               "kk_xlbomd_update")
        return out

    def profile_enable(self, on: bool = True):
        _check(LIB.kk_profile_enable(self._h, 1 if on else 0), "kk_profile_enable")

    def profile_reset(self):
        _check(LIB.kk_profile_reset(self._h), "kk_profile_reset")

    def profile_read(self, kernel_id: int):
        ms, cnt = ctypes.c_double(), ctypes.c_int()
        _check(LIB.kk_profile_read(self._h, kernel_id, ctypes.byref(ms), ctypes.byref(cnt)), "kk_profile_read")
        return ms.value, cnt.value


class Batch:
    """Many independent systems updated together (krylov_kernel_apply_batch)."""

    def __init__(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._b = ctypes.c_void_p()
        _check(LIB.kk_batch_create(ctypes.byref(self._b), ctypes.c_void_p(stream.cuda_stream)), "kk_batch_create")
        self.n_atoms = []
        self._keep = []

    def close(self):
        if self._b:
            _check(LIB.kk_batch_destroy(self._b), "kk_batch_destroy")
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, systems, precision: int = KK_FP64):
        """systems: list of dicts with offsets (host ints), S, Z, Q_up, Q_dn, eps_up, eps_dn,
        gamma (device float64 tensors), W, kT, n_electrons."""
        ns = len(systems)
        offs = [np.ascontiguousarray(np.asarray(s["offsets"], dtype=np.int32)) for s in systems]
        n_atoms = (ctypes.c_int * ns)(*[len(o) - 1 for o in offs])
        off_ptrs = (ctypes.c_void_p * ns)(*[o.ctypes.data for o in offs])

        def table(key):
            return (ctypes.c_void_p * ns)(*[_dev(s[key], key).value for s in systems])

        def vals(key):
            return (ctypes.c_double * ns)(*[float(s[key]) for s in systems])

        tabs = [table(k) for k in ("S", "Z", "Q_up", "Q_dn", "eps_up", "eps_dn", "gamma")]
        _check(LIB.kk_batch_prepare(self._b, ns, n_atoms, off_ptrs, *tabs, vals("W"), vals("kT"),
                                    vals("n_electrons"), int(precision)), "kk_batch_prepare")
        self.n_atoms = [len(o) - 1 for o in offs]
        return self

    def krylov_kernel_apply(self, deltas, m: int, outs=None, info: bool = True):
        import torch
        ns = len(self.n_atoms)
        if outs is None:
            outs = [torch.empty_like(d) for d in deltas]
        dt = (ctypes.c_void_p * ns)(*[_dev(d, "delta", 2 * n).value for d, n in zip(deltas, self.n_atoms)])
        ot = (ctypes.c_void_p * ns)(*[_dev(o, "Kdelta", 2 * n).value for o, n in zip(outs, self.n_atoms)])
        if info:
            inf = (KKInfo * ns)()
            _check(LIB.krylov_kernel_apply_batch(self._b, dt, int(m), ot, inf), "krylov_kernel_apply_batch",
                   ok=(KK_OK, KK_BREAKDOWN, KK_ESINGULAR))
            return outs, [KrylovInfo(x.rank_used, x.status, x.min_pivot, x.max_pivot, x.ls_residual) for x in inf]
        _check(LIB.krylov_kernel_apply_batch(self._b, dt, int(m), ot, None), "krylov_kernel_apply_batch")
        return outs, None

    def set_tuning(self, small_np_max: int, workgroups_per_cu: int):
        """Fix the tile-class threshold and persistent workgroups per CU (no autotuning)."""
        _check(LIB.kk_batch_set_tuning(self._b, int(small_np_max), int(workgroups_per_cu)), "kk_batch_set_tuning")
        return self

    def tuning(self):
        a, g, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(LIB.kk_batch_tuning(self._b, ctypes.byref(a), ctypes.byref(g), ctypes.byref(ms)), "kk_batch_tuning")
        return dict(small_np_max=a.value, workgroups_per_cu=g.value, update_ms=ms.value)
