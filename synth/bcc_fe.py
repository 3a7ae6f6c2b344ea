"""Seeded synthetic bcc-Fe tight-binding systems.

This module only draws and assembles model inputs: positions, the
charge-independent Hamiltonian H0, the overlap S, the screened Coulomb
matrix gamma, the Stoner constant W, a reference expansion point n_ref and a
residual vector delta. It contains none of the Krylov-kernel or
response arithmetic; the oracle and the HIP path both start from its output.

The paper's Fe parameterization (PLATO Slater-Koster tables, Hubbard U,
Stoner J_l, repulsive pair potential; Sec. III.D) is not printed, so the
numbers below are a stand-in with the paper's system type: a periodic bcc Fe
supercell with 9 s/p/d orbitals per atom, ferromagnetic expansion point,
electronic temperature kT = 0.25 eV (Sec. III.B describes the 16-atom bcc
supercell used there).

Recipe (all energies in eV, lengths in Angstrom unless stated):
  * bcc lattice, a = 2.87, n_c^3 conventional cells, atoms ordered by cell
    (ix, iy, iz) lexicographically, then basis site (0,0,0), (1/2,1/2,1/2).
  * displacements: each Cartesian component iid N(0, 0.05).
  * onsite: diag(s=-4.0, p=+2.0 x3, d=-8.5 x5) + iid N(0, 0.1) per orbital.
  * hopping: for every unordered pair I<J (row-major upper-triangle order) a
    symmetric 9x9 block B_IJ with iid N(0,1) upper triangle (incl. diagonal,
    row-major order); H_IJ = 1.5 * B_IJ * w_IJ with
    w_IJ = sum over periodic images with r < 5 of exp(-(r - 2.48)/0.6).
    Blocks are drawn for every pair, in range or not, so the random stream
    does not depend on the geometry.
  * overlap: independent blocks B'_IJ with the same weights w_IJ form X;
    S = I + s_scale * X / rho(X), rho = spectral radius, so eig(S) lies in
    [1 - s_scale, 1 + s_scale] (SPD for s_scale < 1). rho is taken from a
    dense symmetric eigensolve for small systems and from Lanczos (ARPACK,
    fixed start vector) above 2048 basis functions.
  * gamma_IJ = 1 / sqrt(r^2 + U^-2) Hartree with r in Bohr (minimum image when
    periodic), gamma_II = U, U = 0.4 Hartree; converted to eV.
  * W = -0.015 Hartree (one Stoner constant for all atoms and shells).
  * N_e = 8 valence electrons per atom over both spins.
  * delta (charge then magnetization, length 2N): iid N(0, 0.01).
  * expansion point n_ref = (n_q, n_m): neutral atoms n_q = 0 and moments
    n_m = 2.2 + iid N(0, 0.1) per atom, so that the two spin Hamiltonians have
    different eigenvectors (a uniform moment would only shift the spectrum
    rigidly). Random charges are avoided because the unscreened gamma turns
    them into onsite potentials of several eV in large cells.
  Draw order from numpy PCG64 default_rng(seed): displacements, onsite,
  H blocks, S blocks, delta, n_m.

Clusters (open boundaries) take the n sites of an 8x8x8-cell bcc lattice
nearest its centre (ties broken by site index) and use no images.
"""

from __future__ import annotations

import numpy as np

HARTREE_EV = 27.211386
BOHR_ANG = 0.52917721
A_LATTICE = 2.87
ORBITALS_PER_ATOM = 9
ONSITE_EV = np.array([-4.0, 2.0, 2.0, 2.0, -8.5, -8.5, -8.5, -8.5, -8.5])
HOP_SCALE_EV = 1.5
R0 = 2.48
DECAY = 0.6
CUTOFF = 5.0
U_HARTREE = 0.4
W_HARTREE = -0.015
KT_EV = 0.25
ELECTRONS_PER_ATOM = 8


def bcc_sites(n_c: int) -> np.ndarray:
    """Ideal bcc sites of an n_c^3 conventional-cell supercell, shape (2 n_c^3, 3)."""
    idx = np.arange(n_c)
    cells = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1).reshape(-1, 3)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    return (A_LATTICE * (cells[:, None, :] + basis[None, :, :])).reshape(-1, 3)


def cluster_sites(n_atoms: int, n_c: int = 8) -> np.ndarray:
    """The n_atoms sites of an n_c^3-cell bcc lattice nearest its centre."""
    sites = bcc_sites(n_c)
    centre = sites.mean(axis=0)
    d2 = ((sites - centre) ** 2).sum(axis=1)
    order = np.lexsort((np.arange(len(sites)), d2))  # distance, then site index
    return sites[np.sort(order[:n_atoms])]


def _sym_blocks(vals: np.ndarray) -> np.ndarray:
    """(P, 45) upper-triangle values -> (P, 9, 9) symmetric blocks."""
    iu0, iu1 = np.triu_indices(ORBITALS_PER_ATOM)
    blk = np.zeros((vals.shape[0], ORBITALS_PER_ATOM, ORBITALS_PER_ATOM))
    blk[:, iu0, iu1] = vals
    blk[:, iu1, iu0] = vals
    return blk


def _shifts(periodic: bool) -> np.ndarray:
    if not periodic:
        return np.zeros((1, 3))
    s = np.arange(-1, 2)
    return np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3).astype(float)


def _spectral_radius(x: np.ndarray) -> float:
    if not np.any(x):
        return 0.0
    if x.shape[0] <= 2048:
        ev = np.linalg.eigvalsh(x)
        return float(max(abs(ev[0]), abs(ev[-1])))
    from scipy.sparse.linalg import eigsh
    val = eigsh(x, k=1, which="LM", v0=np.ones(x.shape[0]), tol=1e-13,
                return_eigenvectors=False)
    return float(abs(val[0]))


def make_system(n_cells: int | None = None, *, n_atoms: int | None = None, seed: int,
                s_scale: float = 0.15, periodic: bool | None = None,
                uniform_moment: bool = False) -> dict:
    """Build one synthetic Fe system.

    Give either n_cells (periodic supercell of 2 n_cells^3 atoms) or n_atoms
    (open cluster). Returns a dict of float64 numpy arrays and scalars:
      H0 (Nb,Nb), S (Nb,Nb), gamma (N,N), W, kT, n_electrons, valence (N,)
      (neutral-atom electron counts, the Mulliken reference), offsets (N+1,),
      positions (N,3), delta (2N,), n_ref (2N,), box (L or None),
      r2_bohr (N,N) squared minimum-image distances in Bohr^2 (zero diagonal),
      U (eV) and hartree_ev, with which gamma can be rebuilt at another U.
    uniform_moment=True replaces n_ref by (0, 2.2) for every atom.
    """
    if (n_cells is None) == (n_atoms is None):
        raise ValueError("give exactly one of n_cells, n_atoms")
    if n_cells is not None:
        sites = bcc_sites(n_cells)
        box = A_LATTICE * n_cells
        periodic = True if periodic is None else periodic
    else:
        sites = cluster_sites(n_atoms)
        box = None
        periodic = False
    n = len(sites)
    nb = n * ORBITALS_PER_ATOM
    rng = np.random.default_rng(seed)

    pos = sites + rng.normal(0.0, 0.05, size=(n, 3))
    onsite = ONSITE_EV[None, :] + rng.normal(0.0, 0.1, size=(n, ORBITALS_PER_ATOM))
    iu_i, iu_j = np.triu_indices(n, k=1)
    hvals = rng.standard_normal((iu_i.size, 45))
    svals = rng.standard_normal((iu_i.size, 45))
    delta = rng.normal(0.0, 0.01, size=2 * n)
    n_q = np.zeros(n)
    n_m = 2.2 + rng.normal(0.0, 0.1, size=n)
    if uniform_moment:
        n_q = np.zeros(n)
        n_m = np.full(n, 2.2)

    # Pair weights summed over images within the cutoff.
    diff = pos[None, :, :] - pos[:, None, :]
    if periodic:
        diff -= box * np.round(diff / box)  # bring into (-L/2, L/2]
    weight = np.zeros((n, n))
    rmin2 = np.full((n, n), np.inf)
    for s in _shifts(periodic):
        d = diff + (box * s if periodic else 0.0)
        r = np.sqrt((d ** 2).sum(axis=-1))
        np.minimum(rmin2, r ** 2, out=rmin2)
        weight += np.where(r < CUTOFF, np.exp(-(r - R0) / DECAY), 0.0)
    np.fill_diagonal(weight, 0.0)

    w_pair = weight[iu_i, iu_j]
    act = np.nonzero(w_pair > 0.0)[0]
    ai, aj = iu_i[act], iu_j[act]

    def assemble(blocks: np.ndarray, scale: float) -> np.ndarray:
        m4 = np.zeros((n, ORBITALS_PER_ATOM, n, ORBITALS_PER_ATOM))
        b = blocks * (scale * w_pair[act])[:, None, None]
        m4[ai, :, aj, :] = b
        m4[aj, :, ai, :] = np.transpose(b, (0, 2, 1))
        return m4.reshape(nb, nb)

    H0 = assemble(_sym_blocks(hvals[act]), HOP_SCALE_EV)
    H0[np.diag_indices(nb)] = onsite.reshape(-1)
    X = assemble(_sym_blocks(svals[act]), 1.0)
    rho = _spectral_radius(X)
    S = np.eye(nb) + (s_scale / rho) * X if rho > 0 else np.eye(nb)

    rb2 = rmin2 / BOHR_ANG ** 2
    gamma = HARTREE_EV / np.sqrt(rb2 + 1.0 / U_HARTREE ** 2)
    np.fill_diagonal(gamma, U_HARTREE * HARTREE_EV)
    np.fill_diagonal(rb2, 0.0)

    return dict(
        H0=H0, S=S, gamma=gamma, W=W_HARTREE * HARTREE_EV, kT=KT_EV,
        n_electrons=float(ELECTRONS_PER_ATOM * n),
        valence=np.full(n, float(ELECTRONS_PER_ATOM)),
        offsets=np.arange(0, nb + 1, ORBITALS_PER_ATOM, dtype=np.int32),
        positions=pos, delta=delta, n_ref=np.concatenate([n_q, n_m]),
        box=box, n_atoms=n, n_basis=nb, seed=seed,
        r2_bohr=rb2, U=U_HARTREE * HARTREE_EV, hartree_ev=HARTREE_EV,
    )


def cluster_sizes(count: int = 64, seed: int = 64, lo: int = 16, hi: int = 250) -> np.ndarray:
    """Atom counts of the uneven-cluster batch, uniform in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, count)


def krylov_vectors(n_atoms: int, count: int, seed: int) -> np.ndarray:
    """(count, 2N) iid N(0,1) direction vectors for response tests."""
    return np.random.default_rng(seed).standard_normal((count, 2 * n_atoms))


def gradient_direction(sysd: dict, seed: int) -> dict:
    """A seeded direction in (delta, U, W, H0) for directional-derivative checks.

    delta: iid N(0, 1e-2) per entry; U and W: 10 % of their values; H0: a
    symmetric matrix (E + E^T) / (2 sqrt(Nb)) with E iid N(0, 1), drawn in that
    order from default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    nb = sysd["n_basis"]
    dd = rng.standard_normal(2 * sysd["n_atoms"]) * 1e-2
    E = rng.standard_normal((nb, nb))
    dH = 0.5 * (E + E.T) / np.sqrt(nb)
    return dict(delta=dd, U=0.1 * sysd["U"], W=0.1 * abs(sysd["W"]), H0=dH)


def symmetric_direction(nb: int, seed: int) -> np.ndarray:
    """(E + E^T) / (2 sqrt(Nb)), E iid N(0, 1) from default_rng(seed): a probe for matrix gradients."""
    E = np.random.default_rng(seed).standard_normal((nb, nb))
    return 0.5 * (E + E.T) / np.sqrt(nb)
