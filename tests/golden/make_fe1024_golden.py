"""Write the FP64 oracle's results for the 1024-atom bcc-Fe workload.

Calls only the oracle (and the seeded input generator). The GPU tests
compare the HIP path, prepared from an independent device eigensolve, with
these values; only quantities that do not depend on the eigenvector basis
(responses, the kernel result, mu) are stored.

Usage: python tests/golden/make_fe1024_golden.py   (about 10-20 min on 8 cores)
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

CELLS, SEED, RANK, VSEED = 8, 1024, 12, 4242


def main():
    t0 = time.time()
    sysd = make_system(CELLS, seed=SEED)
    ep = expansion_point(sysd)
    print(f"expansion point {time.time() - t0:.0f} s, mu = {ep['mu']:.15f}", flush=True)
    v = krylov_vectors(sysd["n_atoms"], 1, VSEED)[0]
    q1 = response(sysd, ep, v)
    print(f"response {time.time() - t0:.0f} s", flush=True)
    kd, parts = kernel_apply(sysd, ep, sysd["delta"], RANK, return_parts=True)
    print(f"kernel {time.time() - t0:.0f} s, rank {parts['rank']}", flush=True)
    out = dict(
        description="FP64 oracle at the 1024-atom bcc-Fe workload (synth.make_system(8, seed=1024)); "
                    "q1 = response to v = synth.krylov_vectors(1024, 1, 4242)[0]; "
                    "Kdelta = rank-12 Krylov kernel applied to the system's delta with K0 = -I",
        cells=CELLS, seed=SEED, rank=RANK, v_seed=VSEED, mu=ep["mu"],
        q1=q1.tolist(), Kdelta=kd.tolist(), rank_used=int(parts["rank"]),
        gram_eigs=np.linalg.eigvalsh(parts["O"]).tolist(),
    )
    with open(os.path.join(HERE, "fe1024_oracle.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote golden in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
