"""Mulliken projection of a spin density-matrix change.

Test infrastructure (see the package docstring).

Sec. III.A: the Mulliken charge of atom I sums (D - D0)_ij S_ji over its
orbitals i and all j, over both spins; the spin moment takes up minus down.
For a change dD^sigma the D0 term is absent.
"""

from __future__ import annotations

import numpy as np


def mulliken(dD_up: np.ndarray, dD_dn: np.ndarray, S: np.ndarray, offsets) -> np.ndarray:
    """(dq, dm) of length 2N from the two spin density-matrix changes."""
    off = np.asarray(offsets)
    natoms = len(off) - 1
    dn = []
    for dD in (dD_up, dD_dn):
        pop = np.zeros(natoms)
        for a in range(natoms):
            for i in range(off[a], off[a + 1]):
                pop[a] += float(np.dot(dD[i, :], S[:, i]))
        dn.append(pop)
    return np.concatenate([dn[0] + dn[1], dn[0] - dn[1]])
