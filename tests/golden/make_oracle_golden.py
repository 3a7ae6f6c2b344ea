"""Write the FP64 oracle's results for the large bcc-Fe workloads.

Calls only the oracle (and the seeded input generator). The GPU tests
compare the HIP path, prepared from an independent device eigensolve, with
these values; only quantities that do not depend on the eigenvector basis
(responses, the kernel result, mu) are stored.

  fe1024: 8x8x8 cells, seed 1024, rank 12, one response   (about 10-20 min on 8 cores)
  fe432:  6x6x6 cells, seed 432,  rank 8,  eight responses (about 3-5 min on 8 cores)

Usage: python tests/golden/make_oracle_golden.py fe1024|fe432
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
from synth import make_system, krylov_vectors  # noqa: E402

WORKLOADS = {
    # name: (cells, seed, rank, v_seed, number of fixed response directions)
    "fe1024": (8, 1024, 12, 4242, 1),
    "fe432": (6, 432, 8, 4343, 8),
}


def main(name):
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
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote golden in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "fe1024")
