"""Throughput of the rank-m spin-charge Krylov kernel update on one MI355X.

One step = one krylov_kernel_apply: m sequential density-matrix responses
(potentials, forward eigenbasis transform with the Fermi Hadamard product and
chemical-potential shift, back-transform with the Mulliken projection) plus
the Krylov orthogonalization and the m x m Gram solve, on a prepared
1024-atom bcc-Fe system (Nb = 9216, m = 12, FP64). Inputs are resident in
HBM before the timed region.

Prints one JSON line. The roofline object reports the dominant transform
kernel: algorithmic flops per launch (2 spins x 2 Nb^3) over its average
launch time from HIP events recorded by the library on the launch stream.
The cpu_baseline leg times the plain FP64 oracle on the host for a bounded
sample of the same workload (one of the m responses of an update).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
FP16_MFMA_PEAK_TFLOPS = 2500.0  # dense; the split form spends three FP16 products per FP64 product
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=8, help="bcc supercell edge in cells (2 n^3 atoms)")
    ap.add_argument("--rank", type=int, default=12)
    ap.add_argument("--seed", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="transform arithmetic: FP64 MFMA, or FP16 x 3 split products")
    ap.add_argument("--traffic-file", default=None,
                    help="HBM traffic summary of the dominant kernel (default: profiles/traffic_<precision>_1024.json)")
    ap.add_argument("--workload", choices=["fe1024", "clusters64", "fe1024grad"], default="fe1024",
                    help="fe1024: one 1024-atom bcc cell (headline); clusters64: 64 uneven open clusters, "
                         "16-250 atoms, rank 6, batched in one graph launch; fe1024grad: K delta and its "
                         "reverse pass (gradients of ||K delta||^2) on the 1024-atom cell")
    ap.add_argument("--grad-wrt", choices=["all", "delta"], default="all",
                    help="fe1024grad: gradients with respect to delta, gamma, W and H (all) or without the "
                         "expansion-point part (delta: delta, gamma, W only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB elementwise copy kernel 3 times (scales HBM counters)")
    return ap.parse_args()


def gemm_source_digest(precision: str = "fp64") -> str:
    """First 16 hex of the sha256 of the header holding the transform kernels."""
    import hashlib
    name = "kk_gemm.hpp" if precision == "fp64" else "kk_gemm_mixed.hpp"
    src = os.path.join(ROOT, "paper_2303_03529_amd", "csrc", name)
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def cpu_baseline(sysd, m):
    """Oracle timed on the host: one response (one of m directions) at full size."""
    import numpy as np

    from oracle.expansion import congruence_cholesky, expansion_point
    from oracle.response import response

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    ep = expansion_point(sysd, Z=congruence_cholesky(sysd["S"]))
    v = np.random.default_rng(7).standard_normal(2 * sysd["n_atoms"])
    v /= np.linalg.norm(v)
    t0 = time.perf_counter()
    response(sysd, ep, v)
    dt = time.perf_counter() - t0
    return {
        "value": 1.0 / (m * dt),
        "unit": "updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"one oracle response (1 of the m={m} Krylov directions of one update, both spins, "
                  f"{sysd['n_atoms']} atoms) timed once: {dt:.2f} s; value = 1/(m x that time)",
    }


def bench_clusters(args):
    """Batched form: 64 uneven clusters (atom counts uniform in [16, 250], seeds 10000+i),
    rank 6, one graph launch per batched update."""
    import numpy as np
    import torch

    from paper_2303_03529_amd import krylov
    from paper_2303_03529_amd.caller_setup import DeviceSystem
    from synth import cluster_sizes, make_system

    dev = "cuda:0"
    m = 6 if args.rank == 12 else args.rank
    prec = krylov.KK_MIXED_F16 if args.precision == "mixed" else krylov.KK_FP64
    t_setup = time.perf_counter()
    sizes = [int(x) for x in cluster_sizes(64, seed=64)]
    systems, deltas, nbs = [], [], []
    for i, n in enumerate(sizes):
        sysd = make_system(n_atoms=n, seed=10_000 + i)
        e = DeviceSystem(sysd, dev).expansion()
        systems.append(dict(offsets=sysd["offsets"], S=e["S"], Z=e["Z"], Q_up=e["Q_up"], Q_dn=e["Q_dn"],
                            eps_up=e["eps_up"], eps_dn=e["eps_dn"], gamma=e["gamma"], W=sysd["W"], kT=sysd["kT"],
                            n_electrons=sysd["n_electrons"]))
        deltas.append(torch.as_tensor(sysd["delta"], dtype=torch.float64, device=dev))
        nbs.append(sysd["n_basis"])
    b = krylov.Batch().prepare(systems, prec)
    del systems
    torch.cuda.empty_cache()
    outs = [torch.empty_like(d) for d in deltas]
    print(f"# setup {time.perf_counter() - t_setup:.1f} s (64 clusters, {min(sizes)}-{max(sizes)} atoms, m={m})",
          file=sys.stderr, flush=True)
    _, infos = b.krylov_kernel_apply(deltas, m, outs)          # autotune + capture
    for _ in range(args.warmup):
        b.krylov_kernel_apply(deltas, m, outs, info=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.krylov_kernel_apply(deltas, m, outs, info=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tune = b.tuning()
    b.close()
    flops = sum(8.0 * m * nb ** 3 for nb in nbs)
    peak = FP64_MFMA_PEAK_TFLOPS if prec == krylov.KK_FP64 else FP16_MFMA_PEAK_TFLOPS / 3.0
    tflops = flops / (elapsed / args.steps) / 1e12
    res = {
        "metric": "batched Krylov rank-m kernel updates/sec, 64 uneven Fe clusters",
        "value": args.steps / elapsed, "unit": "batch updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == krylov.KK_FP64 else "f16x3+f64", "data": "synthetic",
        "config": {"workload": f"64 open bcc-Fe clusters, atoms {min(sizes)}-{max(sizes)}, rank m={m}, "
                               "one hipGraph launch per batched update, autotuned tiles",
                   "systems": 64, "rank": m, "atoms_total": sum(sizes)},
        "system_updates_per_s": 64 * args.steps / elapsed,
        "update_tflops": tflops, "mfma_frac_update": tflops / peak, "peak_tflops": peak,
        "tuning": tune, "ranks_used": sorted(set(i.rank_used for i in infos)),
    }
    print(json.dumps(res), flush=True)


def bench_grad(args):
    """Differentiation form: one step = krylov_kernel_apply plus krylov_kernel_adjoint (reusing
    the expansion) for L = ||K delta||^2 on the prepared 1024-atom system, FP64."""
    import torch

    from paper_2303_03529_amd import krylov
    from paper_2303_03529_amd.caller_setup import expansion_point_device
    from synth import make_system

    dev = "cuda:0"
    t_setup = time.perf_counter()
    sysd = make_system(args.cells, seed=args.seed)
    N, nb, m = sysd["n_atoms"], sysd["n_basis"], args.rank
    e = expansion_point_device(sysd, dev)
    h = krylov.Handle()
    prec = krylov.KK_FP64 if args.precision == "fp64" else krylov.KK_MIXED_F16
    h.prepare(sysd["offsets"], e["S"], e["Z"], e["Q_up"], e["Q_dn"], e["eps_up"], e["eps_dn"],
              e["gamma"], sysd["W"], sysd["kT"], sysd["n_electrons"], prec)
    delta = torch.as_tensor(sysd["delta"], dtype=torch.float64, device=dev)
    out = torch.empty_like(delta)
    ref = None
    if prec != krylov.KK_FP64:  # FP64 gradient on the same inputs, for the error of the split forward
        h64 = krylov.Handle()
        h64.prepare(sysd["offsets"], e["S"], e["Z"], e["Q_up"], e["Q_dn"], e["eps_up"], e["eps_dn"],
                    e["gamma"], sysd["W"], sysd["kT"], sysd["n_electrons"], krylov.KK_FP64)
        x64, _ = h64.krylov_kernel_apply(delta, m)
        ref = h64.krylov_kernel_adjoint(delta, m, 2.0 * x64, reuse_forward=True,
                                        want_H=args.grad_wrt == "all")
        ref = {k: ref[k].cpu() for k in ("delta", "H_up", "H_dn") if ref[k] is not None}
        h64.close()
        del h64
    del e
    torch.cuda.empty_cache()
    print(f"# setup {time.perf_counter() - t_setup:.1f} s (N={N}, Nb={nb}, m={m})", file=sys.stderr, flush=True)

    want_H = args.grad_wrt == "all"

    def step():
        x, _ = h.krylov_kernel_apply(delta, m, out=out, info=False)
        return h.krylov_kernel_adjoint(delta, m, 2.0 * x, reuse_forward=True, want_H=want_H)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h.profile_enable(True)
    h.profile_reset()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    names = {0: "forward_fermi", 1: "back_mulliken", 2: "reverse_forward_xy", 3: "reverse_accumulate"}
    flops_launch = {0: 4.0 * nb ** 3, 1: 4.0 * nb ** 3, 2: 8.0 * nb ** 3, 3: 8.0 * nb ** 3}
    kern = {}
    for kid, name in names.items():
        ms, n = h.profile_read(kid)
        kern[name] = (ms / max(n, 1), n, flops_launch[kid])
    h.profile_enable(False)
    h.close()
    err = None
    if ref is not None:
        err = {k: float((g[k].cpu() - ref[k]).norm() / ref[k].norm()) for k in ref}
    fwd_peak = FP64_MFMA_PEAK_TFLOPS if prec == krylov.KK_FP64 else FP16_MFMA_PEAK_TFLOPS / 3.0
    dom = max(kern, key=lambda k: kern[k][0] * kern[k][1])
    avg_ms, _, fl = kern[dom]
    achieved = fl / (avg_ms * 1e-3) / 1e12
    dom_peak = fwd_peak if dom in ("forward_fermi", "back_mulliken") else FP64_MFMA_PEAK_TFLOPS
    # forward 8 m Nb^3; reverse per direction: X,Y of four items (8), Mulliken of two (4),
    # accumulation (8); final C E' C^T (8 Nb^3). Without H: one response per direction (8).
    if want_H:
        step_flops = 8.0 * m * nb ** 3 + 20.0 * m * nb ** 3 + 8.0 * nb ** 3
    else:
        step_flops = 16.0 * m * nb ** 3
    res = {
        "metric": "Krylov kernel gradient evaluations/sec (K delta and dL/d(delta, gamma, W"
                  + (", H^sigma" if want_H else "") + "), L = ||K delta||^2) at 1024-atom Fe",
        "value": args.steps / elapsed, "unit": "gradient evaluations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == krylov.KK_FP64 else ("f16x3+f64 forward, f64 reverse" if want_H else "f16x3+f64"),
        "data": "synthetic",
        "config": {"workload": f"bcc Fe {N} atoms ({args.cells}^3 cells), Nb={nb}, rank m={m}, "
                               f"{'FP64' if prec == krylov.KK_FP64 else 'split FP16x3'} forward + "
                               f"{'FP64 reverse pass with H gradients' if want_H else 'reverse pass without H'}, "
                               "K0=-I", "n_atoms": N, "n_basis": nb, "rank": m},
        "step_tflops": step_flops / (elapsed / args.steps) / 1e12,
        "grad_err_vs_fp64": err,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": round(dom_peak, 2),
                     "unit": "TFLOP/s", "frac": round(achieved / dom_peak, 4), "traffic": None,
                     "kernel": dom, "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": fl,
                     "other_kernel_avg_ms": {k: round(v[0], 4) for k, v in kern.items() if k != dom}},
        "grad_norms": {k: float(g[k].norm()) for k in ("delta", "H_up") if g[k] is not None},
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of this path is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2303_03529_amd import krylov
    from paper_2303_03529_amd.caller_setup import expansion_point_device
    from synth import make_system

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.workload == "clusters64":
        return bench_clusters(args)
    if args.workload == "fe1024grad":
        return bench_grad(args)
    t_setup = time.perf_counter()
    sysd = make_system(args.cells, seed=args.seed)
    N, nb, m = sysd["n_atoms"], sysd["n_basis"], args.rank
    e = expansion_point_device(sysd, dev)
    prec = krylov.KK_FP64 if args.precision == "fp64" else krylov.KK_MIXED_F16
    h = krylov.Handle()
    h.prepare(sysd["offsets"], e["S"], e["Z"], e["Q_up"], e["Q_dn"], e["eps_up"], e["eps_dn"],
              e["gamma"], sysd["W"], sysd["kT"], sysd["n_electrons"], prec)
    ref = None
    if prec != krylov.KK_FP64:
        # FP64 path on the same prepared inputs, for the error of the split-precision form
        h64 = krylov.Handle()
        h64.prepare(sysd["offsets"], e["S"], e["Z"], e["Q_up"], e["Q_dn"], e["eps_up"], e["eps_dn"],
                    e["gamma"], sysd["W"], sysd["kT"], sysd["n_electrons"], krylov.KK_FP64)
        d64 = torch.as_tensor(sysd["delta"], dtype=torch.float64, device=dev)
        ref, _ = h64.krylov_kernel_apply(d64, args.rank)
        ref = ref.cpu().numpy()
        h64.close()
        del h64
    del e
    torch.cuda.empty_cache()
    delta = torch.as_tensor(sysd["delta"], dtype=torch.float64, device=dev)
    out = torch.empty_like(delta)
    setup_s = time.perf_counter() - t_setup
    print(f"# setup {setup_s:.1f} s (N={N}, Nb={nb}, m={m})", file=sys.stderr, flush=True)

    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    for _ in range(args.warmup):
        h.krylov_kernel_apply(delta, m, out=out, info=False)
    torch.cuda.synchronize()
    h.profile_enable(True)
    h.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h.krylov_kernel_apply(delta, m, out=out, info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_fwd, n_fwd = h.profile_read(0)
    ms_back, n_back = h.profile_read(1)
    h.profile_enable(False)
    _, info = h.krylov_kernel_apply(delta, m, out=out, info=True)
    assert info.rank_used == m, info
    err_vs_fp64 = None
    if ref is not None:
        err_vs_fp64 = float(np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref))

    elapsed = t1 - t0
    value = args.steps / elapsed
    flops_launch = 2 * 2.0 * nb ** 3  # one transform, both spins
    kernels = {
        "forward_fermi": (ms_fwd / max(n_fwd, 1), n_fwd),
        "back_mulliken": (ms_back / max(n_back, 1), n_back),
    }
    dom = max(kernels, key=lambda k: kernels[k][0] * kernels[k][1])
    avg_ms = kernels[dom][0]
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12
    traffic = None
    traffic_file = args.traffic_file or os.path.join(ROOT, "profiles", f"traffic_{args.precision}_1024.json")
    if os.path.exists(traffic_file):
        tr = json.load(open(traffic_file))
        if (tr.get("kernel") == dom and tr.get("n_basis") == nb
                and tr.get("source_digest") == gemm_source_digest(args.precision)):
            traffic = tr.get("bytes_per_launch")
    peak = FP64_MFMA_PEAK_TFLOPS if prec == krylov.KK_FP64 else FP16_MFMA_PEAK_TFLOPS / 3.0
    roofline = {
        "bound": "mfma", "achieved": round(achieved, 3), "peak": round(peak, 2),
        "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
        "kernel": dom, "avg_launch_ms": round(avg_ms, 4),
        "flops_per_launch": flops_launch,
        "other_kernel_avg_ms": {k: round(v[0], 4) for k, v in kernels.items() if k != dom},
    }
    update_flops = 8.0 * m * nb ** 3
    res = {
        "metric": "Krylov rank-m kernel updates/sec at 1024-atom Fe",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == krylov.KK_FP64 else "f16x3+f64",
        "data": "synthetic",
        "config": {"workload": f"bcc Fe {N} atoms ({args.cells}^3 cells), Nb={nb}, rank m={m}, "
                               f"{'FP64' if prec == krylov.KK_FP64 else 'split FP16x3'} transforms, K0=-I",
                   "n_atoms": N, "n_basis": nb, "rank": m, "seed": args.seed},
        "update_tflops": update_flops / (elapsed / args.steps) / 1e12,
        "mfma_util_update": update_flops / (elapsed / args.steps) / 1e12 / peak,
        "err_vs_fp64": err_vs_fp64,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    h.close()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(sysd, m)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
