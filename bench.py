#!/usr/bin/env python3
"""Benchmark of the per-time-step update on one MI355X.

Default workload: D3Q19 128^3 periodic binary slab (PR EOS, BGK tau = 0.8,
FP32 populations with FP64 EOS logarithms), the HBM-bound workload of the
metric.  A step is one pass of the whole update (moments + EOS, force +
collision + streaming) over every node; inputs are resident in HBM before the
timed region.

Prints ONE JSON line: component-MLUPS of the whole job, the roofline of the
dominant kernel (algorithmic bytes per launch / average launch duration, HIP
events on the solver's stream), and the FP64 oracle timed on the host cores on
a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2212_10680_amd import fuglbm as F  # noqa: E402
from paper_2212_10680_amd import workloads as wl  # noqa: E402

METRIC = "component-MLUPS & HBM-BW fraction; batched VLE solves/s + p99 time-to-equil"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_2212_10680_amd/csrc/kernels.hip", "paper_2212_10680_amd/csrc/device.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(w, precision):
    """Algorithmic HBM bytes per node of each kernel of one step.

    k_moments_eos: read every population, write rho~_i and ln f_i (FP64).
    k_collide_stream: read and write every population, read rho~_i and ln f_i
    once (the stencil re-reads are cache traffic), read and write the previous
    force sum (D FP64).  The FP32 form also reads the rest-population reference.
    """
    Q = 9 if w.lattice == "D2Q9" else 19
    D = w.D
    nc = w.ncomp
    s = 8 if precision == "fp64" else 4
    ref = 0 if precision == "fp64" else 4 * nc
    pops = Q * nc * s
    k1 = pops + ref + 2 * 8 * nc
    k2 = 2 * pops + ref + 2 * 8 * nc + 2 * s * D
    # per-node-step figure: populations once in and out, the FP64 densities and
    # ln f once each way, the force history (population precision) once each way
    step = 2 * pops + 32 * nc + 2 * s * D
    return {"k_moments_eos": k1, "k_collide_stream": k2, "step": step}


def stored_traffic(kernel, nodes):
    """HBM bytes per launch from the committed PMC counters, if they were taken
    on the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k or k.get("nodes") != nodes:
        return None
    return k.get("bytes_per_launch")


def cpu_baseline(w, budget_s=15.0):
    """FP64 oracle (as it stands) on a bounded slice of the workload."""
    from oracle import lbm
    from oracle import thermo as th

    comps, kij, T = w.thermo()
    mix = th.Mixture([c["Tc"] for c in comps], [c["Pc"] for c in comps], [c["omega"] for c in comps],
                     T, kij=kij, M=[c["M"] for c in comps], kappa=[c["kappa"] for c in comps])
    if w.D == 3:
        shape = (w.shape[0], 32, 32)
    else:
        shape = (w.shape[0], min(w.shape[1], 64))
    ws = w.scaled(shape)
    ws.radius, ws.separation = w.radius, w.separation
    rho, u = wl.initial_field(ws)
    o = lbm.OracleLBM(mix, w.lattice, shape, tau=w.tau, collision=w.collision)
    o.init(rho.reshape(w.ncomp, -1), None if u is None else u.reshape(w.D, -1))
    o.run(1)  # warm-up
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.run(1)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= 10000:
            break
    dt = time.perf_counter() - t0
    nodes = int(np.prod(shape))
    return {"value": round(nodes * w.ncomp * steps / dt / 1e6, 3), "unit": "component-MLUPS",
            "cores": lbm.num_threads(), "kind": "oracle",
            "sample": f"{w.lattice} {'x'.join(map(str, shape))} slice of the workload, {steps} steps, "
                      f"FP64, {w.collision}, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="binary_slab_3d", choices=sorted(wl.WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (PMC byte-counter scale)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU; runs on more than one GPU are not part of it",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    F.load()  # fails loudly when the HIP library is not built

    w = wl.WORKLOADS[args.workload]
    precision = args.precision or w.precision
    p = F.Params.from_workload(w, precision=precision)
    solver = F.Solver(p)
    rho, u = wl.initial_field(w)
    solver.set_state(rho, u)
    print(f"[bench] {w.name} {w.lattice} {w.shape} nc={w.ncomp} {w.collision} tau={w.tau} {precision}",
          file=sys.stderr, flush=True)

    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        gbps = 3 * 2 * 4 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
        print(f"[bench] copy calibration: 4 x {4 * n} bytes read + written; "
              f"copy bandwidth {gbps:.0f} GB/s (read + write)", file=sys.stderr, flush=True)
        del a, b

    solver.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = solver.step_timed(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    nodes = w.nodes
    ms_per_step = 1e3 * wall / args.steps
    value = nodes * w.ncomp * args.steps / wall / 1e6
    ab = algorithmic_bytes(w, precision)
    dominant = max(kms, key=kms.get)
    avg_ms = kms[dominant] / args.steps
    achieved = ab[dominant] * nodes / (avg_ms * 1e-3) / 1e9
    step_gpu_ms = sum(kms.values()) / args.steps
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": stored_traffic(dominant, nodes),
        "kernel": dominant,
        "kernel_avg_ms": round(avg_ms, 4),
        "algorithmic_bytes_per_node": ab[dominant],
        "kernel_ms_per_step": {k: round(v / args.steps, 4) for k, v in kms.items()},
        "step_effective_GBps": round(ab["step"] * nodes / (step_gpu_ms * 1e-3) / 1e9, 1),
        "step_effective_frac": round(ab["step"] * nodes / (step_gpu_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "step_bytes_per_node": ab["step"],
    }
    mass = solver.mass()
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "component-MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 populations / f64 EOS" if precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": w.lattice, "shape": list(w.shape), "ncomp": w.ncomp,
                   "collision": w.collision, "tau": w.tau, "precision": precision,
                   "node_MLUPS": round(nodes * args.steps / wall / 1e6, 1)},
        "roofline": roofline,
        "mass_total": [float(m) for m in mass],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
