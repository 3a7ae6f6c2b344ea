"""Shared set-up for the GPU parity tests: hand identical prepared inputs to
the HIP library and to the oracle."""

from __future__ import annotations

import numpy as np
import torch

DEV = "cuda:0"


def t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def handle_from_expansion(sysd: dict, ep: dict, precision: int = 0):
    """HIP handle prepared with the oracle's own Z, Q, eps (identical inputs)."""
    from paper_2303_03529_amd import krylov
    h = krylov.Handle()
    h.prepare(sysd["offsets"], t(sysd["S"]), t(ep["Z"]), t(ep["Q"][0]), t(ep["Q"][1]),
              t(ep["eps"][0]), t(ep["eps"][1]), t(sysd["gamma"]), sysd["W"], sysd["kT"],
              sysd["n_electrons"], precision)
    return h


def handle_from_device_setup(sysd: dict, precision: int = 0):
    """HIP handle prepared from a device-side eigensolve (independent of the oracle)."""
    from paper_2303_03529_amd import krylov
    from paper_2303_03529_amd.caller_setup import expansion_point_device
    e = expansion_point_device(sysd, DEV)
    h = krylov.Handle()
    h.prepare(sysd["offsets"], e["S"], e["Z"], e["Q_up"], e["Q_dn"], e["eps_up"], e["eps_dn"],
              e["gamma"], sysd["W"], sysd["kT"], sysd["n_electrons"], precision)
    del e
    return h


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
