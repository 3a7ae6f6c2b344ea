"""Write the FP64 oracle's results for the large workloads.

Calls only the oracle (and the seeded input generator). The GPU tests
compare the HIP path, prepared from an independent device eigensolve, with
these values; only quantities that do not depend on the eigenvector basis
(responses, the kernel result, mu, L = ||K delta||^2 and its derivatives)
are stored.

  fe1024:     8x8x8 cells, seed 1024, rank 12, one response      (about 10-20 min on 8 cores)
  fe432:      6x6x6 cells, seed 432,  rank 8,  eight responses   (about 3-5 min on 8 cores)
  clusters64: the 64 open clusters of the batching workload (atom counts
              synth.cluster_sizes(64, 64), system i seeded 10000 + i), rank 6,
              K delta of every system                          (about 5 min on 8 cores)
  fe432grad:  6x6x6 cells, seed 432, rank 8: the oracle gradient (torch.autograd
              through the plain forward of oracle.adjoint) of L = ||K delta||^2 with
              respect to delta, U, W and H0; dL/dH0 is stored through its diagonal,
              its Frobenius norm and its projections on 8 seeded symmetric
              directions; also the size of the dL/dU chain-rule terms
                                                               (about 15 min, ~25 GB)
  fe1024fd:   8x8x8 cells, seed 1024, rank 12: L at theta and at theta +/- h d,
              h = 1e-4, d = synth.gradient_direction(sysd, 11) in (delta, U, W, H0),
              from the oracle's plain forward               (about 40 min on 8 cores)

Usage: python tests/golden/make_oracle_golden.py fe1024|fe432|clusters64|fe432grad|fe1024fd
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.expansion import expansion_point  # noqa: E402
from oracle.krylov import kernel_apply  # noqa: E402
from oracle.response import response  # noqa: E402
from synth import (make_system, krylov_vectors, cluster_sizes, gradient_direction,  # noqa: E402
                   symmetric_direction)

WORKLOADS = {
    # name: (cells, seed, rank, v_seed, number of fixed response directions)
    "fe1024": (8, 1024, 12, 4242, 1),
    "fe432": (6, 432, 8, 4343, 8),
}
CLUSTER_RANK = 6
GRAD432 = dict(cells=6, seed=432, rank=8, h0_dir_seed=5000, h0_dirs=8)
FD1024 = dict(cells=8, seed=1024, rank=12, dir_seed=11, h=1e-4)


def write(name, out, t0):
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote {name} golden in {time.time() - t0:.0f} s", flush=True)


def single(name):
    cells, seed, rank, vseed, nv = WORKLOADS[name]
    t0 = time.time()
    sysd = make_system(cells, seed=seed)
    n = sysd["n_atoms"]
    ep = expansion_point(sysd)
    print(f"expansion point {time.time() - t0:.0f} s, mu = {ep['mu']:.15f}", flush=True)
    vs = krylov_vectors(n, nv, vseed)
    q1 = [response(sysd, ep, v) for v in vs]
    print(f"{nv} responses {time.time() - t0:.0f} s", flush=True)
    kd, parts = kernel_apply(sysd, ep, sysd["delta"], rank, return_parts=True)
    print(f"kernel {time.time() - t0:.0f} s, rank {parts['rank']}", flush=True)
    out = dict(
        description=f"FP64 oracle at the {n}-atom bcc-Fe workload (synth.make_system({cells}, seed={seed})); "
                    f"q1 = responses to v = synth.krylov_vectors({n}, {nv}, {vseed}); "
                    f"Kdelta = rank-{rank} Krylov kernel applied to the system's delta with K0 = -I",
        cells=cells, seed=seed, rank=rank, v_seed=vseed, mu=ep["mu"],
        q1=q1[0].tolist() if nv == 1 else [q.tolist() for q in q1],
        Kdelta=kd.tolist(), rank_used=int(parts["rank"]),
        gram_eigs=np.linalg.eigvalsh(parts["O"]).tolist(),
    )
    write(name, out, t0)


def clusters64():
    t0 = time.time()
    sizes = [int(x) for x in cluster_sizes(64, seed=64)]
    systems = []
    for i, n in enumerate(sizes):
        sysd = make_system(n_atoms=n, seed=10_000 + i)
        ep = expansion_point(sysd)
        kd, parts = kernel_apply(sysd, ep, sysd["delta"], CLUSTER_RANK, return_parts=True)
        systems.append(dict(n_atoms=n, seed=10_000 + i, mu=ep["mu"], Kdelta=kd.tolist(),
                            rank_used=int(parts["rank"]), cond_O=float(np.linalg.cond(parts["O"]))))
        print(f"system {i:2d}: {n:3d} atoms, rank {parts['rank']}, {time.time() - t0:.0f} s", flush=True)
    out = dict(
        description="FP64 oracle for the 64 open bcc-Fe clusters of the batching workload: atom counts "
                    "synth.cluster_sizes(64, seed=64), system i = synth.make_system(n_atoms=n_i, seed=10000 + i); "
                    f"Kdelta = rank-{CLUSTER_RANK} Krylov kernel applied to each system's delta with K0 = -I",
        rank=CLUSTER_RANK, sizes=sizes, systems=systems,
    )
    write("clusters64", out, t0)


def fe432grad():
    from oracle.adjoint import U_gradient_scale, gradients
    t0 = time.time()
    g = GRAD432
    sysd = make_system(g["cells"], seed=g["seed"])
    gr = gradients(sysd, g["rank"])
    print(f"gradients {time.time() - t0:.0f} s, L = {gr['L']:.15e}, rank {gr['rank']}", flush=True)
    GH = gr["H0"]
    proj = []
    for k in range(g["h0_dirs"]):
        E = symmetric_direction(sysd["n_basis"], g["h0_dir_seed"] + k)
        proj.append(float((GH * E).sum()))
    del GH
    u_scale = U_gradient_scale(sysd, g["rank"])
    print(f"U term scale {time.time() - t0:.0f} s: {u_scale:.6e} (dL/dU = {gr['U']:.6e})", flush=True)
    out = dict(
        description=f"FP64 oracle gradient (oracle.adjoint.gradients: torch.autograd through the plain "
                    f"forward) of L = ||K delta||^2, rank {g['rank']}, K0 = -I, at the "
                    f"{sysd['n_atoms']}-atom bcc-Fe workload (synth.make_system({g['cells']}, seed={g['seed']})); "
                    f"dL/dH0 through its diagonal, Frobenius norm and projections sum(G * E_k) on "
                    f"E_k = synth.symmetric_direction(Nb, {g['h0_dir_seed']} + k), k < {g['h0_dirs']}; "
                    "U_term_scale = sum |dL/dgamma_IJ dgamma_IJ/dU| (oracle.adjoint.U_gradient_scale)",
        cells=g["cells"], seed=g["seed"], rank=g["rank"], rank_used=gr["rank"],
        h0_dir_seed=g["h0_dir_seed"], L=gr["L"], Kdelta=gr["Kdelta"].tolist(),
        delta=gr["delta"].tolist(), U=gr["U"], W=gr["W"], H0_diag=np.diag(gr["H0"]).tolist(),
        H0_fro=float(np.linalg.norm(gr["H0"])), H0_proj=proj, U_term_scale=u_scale,
    )
    write("fe432grad", out, t0)


def fe1024fd():
    import torch
    from oracle.adjoint import kernel_loss
    t0 = time.time()
    c = FD1024
    sysd = make_system(c["cells"], seed=c["seed"])
    d = gradient_direction(sysd, c["dir_seed"])
    T = lambda x: torch.as_tensor(np.asarray(x), dtype=torch.float64)  # noqa: E731
    vals = {}
    with torch.no_grad():
        for s in (0.0, c["h"], -c["h"]):
            L = kernel_loss(sysd, T(sysd["delta"] + s * d["delta"]), T(sysd["U"] + s * d["U"]),
                            T(sysd["W"] + s * d["W"]), T(sysd["H0"] + s * d["H0"]), c["rank"])
            vals[s] = float(L)
            print(f"L(theta {s:+.0e} d) = {vals[s]:.16e}  ({time.time() - t0:.0f} s)", flush=True)
    h = c["h"]
    out = dict(
        description=f"FP64 oracle forward (oracle.adjoint.kernel_loss, no autograd) of L = ||K delta||^2, "
                    f"rank {c['rank']}, K0 = -I, at the {sysd['n_atoms']}-atom bcc-Fe workload "
                    f"(synth.make_system({c['cells']}, seed={c['seed']})), at theta = (delta, U, W, H0) and "
                    f"theta +/- h d with h = {h} and d = synth.gradient_direction(sysd, {c['dir_seed']}); "
                    "fd = (L_plus - L_minus) / (2 h) is the oracle's central-difference directional derivative",
        cells=c["cells"], seed=c["seed"], rank=c["rank"], dir_seed=c["dir_seed"], h=h,
        L=vals[0.0], L_plus=vals[h], L_minus=vals[-h], fd=(vals[h] - vals[-h]) / (2 * h),
    )
    write("fe1024fd", out, t0)


if __name__ == "__main__":
    name = sys.argv[1] if len(sys.argv) > 1 else "fe1024"
    {"clusters64": clusters64, "fe432grad": fe432grad, "fe1024fd": fe1024fd}.get(name, lambda: single(name))()
