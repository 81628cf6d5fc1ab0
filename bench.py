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
TIMING_EVERY = 8
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_2212_10680_amd/csrc/kernels.hip", "paper_2212_10680_amd/csrc/device.h",
                  "paper_2212_10680_amd/csrc/launch.h", "paper_2212_10680_amd/build.py"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(w, precision):
    """Algorithmic HBM bytes per node of each kernel of one step.

    k_moments_eos: read every population, write rho~_i, ln f_i and phi (FP64).
    k_collide_stream / k_collide_zmarch (the same work; the second stages the
    FP64 fields through LDS): read and write every population, read rho~_i, ln f_i and
    phi once (the stencil re-reads are cache traffic), read and write the previous
    force sum (D values).  The FP32 form also reads the rest-population reference.
    k_fused_step: the whole step, i.e. the per-node-step figure.
    """
    Q = 9 if w.lattice == "D2Q9" else 19
    D = w.D
    nc = w.ncomp
    s = 8 if precision == "fp64" else 4
    ref = 0 if precision == "fp64" else 4 * nc
    pops = Q * nc * s
    aux = 8 * (2 * nc + 1)          # rho~_i, ln f_i and the interface field phi (FP64)
    k1 = pops + ref + aux
    k2 = 2 * pops + ref + aux + 2 * s * D
    # per-node-step figure: populations once in and out, the FP64 densities,
    # ln f and phi once each way, the force history (population precision) once
    # each way, and the FP32 form's rest-population reference once
    step = 2 * pops + 2 * aux + 2 * s * D + ref
    return {"k_moments_eos": k1, "k_collide_stream": k2, "k_collide_zmarch": k2, "k_fused_step": step,
            "step": step}


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


def serving_bench(n_requests=512, max_steps=50000, pool_mb=256, tick_ms=50.0, plain_subset=16,
                  tol=1e-10, check_every=1000, accuracy_subset=8, policy="largest_first"):
    """Batched VLE serving: FP32-population server vs the plain FP64 path.

    Requests: binary D2Q9 L x 8 slabs, L log-uniform in [64, 2048], feed z1
    redrawn until a S_V = 0.5 state exists; each runs until the rate residual is
    below tol (checked every check_every steps) or max_steps.  Closed loop first
    (all requests present at t = 0) for the saturation throughput, then a
    seeded Poisson stream at 0.8 of it, admitted by the pool budget.
    """
    from paper_2212_10680_amd import serving

    w = wl.WORKLOADS["serving_binary_2d"]
    p32 = F.Params.from_workload(w, precision="fp32")
    reqs, rejected = wl.serving_requests(n=n_requests, seed=0)
    srv = F.Server(p32, pool_bytes=pool_mb << 20, max_slots=512)
    closed = serving.serve(srv, reqs, np.zeros(len(reqs)), tol, check_every, max_steps, tick_ms, policy=policy)
    srv.close()
    print(f"[bench] serving closed loop: {closed['solves_per_s']:.1f} solves/s", file=sys.stderr, flush=True)
    rate = 0.8 * closed["solves_per_s"]
    arrivals = serving.poisson_arrivals(len(reqs), rate, seed=0)
    srv = F.Server(p32, pool_bytes=pool_mb << 20, max_slots=512)
    batched = {}
    opened = serving.serve(srv, reqs, arrivals, tol, check_every, max_steps, tick_ms, policy=policy,
                           on_result=lambda rec, rho: batched.__setitem__(rec["i"], (rho, rec["steps"], rec["status"])))
    srv.close()
    print(f"[bench] serving open loop: {opened['solves_per_s']:.1f} solves/s, "
          f"p99 {opened['p99_latency_s']:.2f} s", file=sys.stderr, flush=True)
    # plain FP64 path (one request at a time, two kernels per step) on a subset
    # spread over the stream, for its throughput; its results against the FP32
    # server at the same step count measure how far the two trajectories drift
    # apart (most of these stop at max_steps, before equilibrium)
    idx = list(range(0, len(reqs), max(1, len(reqs) // plain_subset)))[:plain_subset]
    p64 = F.Params.from_workload(w, precision="fp64")
    times, diffs, psteps = [], [], []
    for i in idx:
        rho, steps, res, conv, dt = serving.solve_plain(p64, reqs[i], tol, check_every, max_steps)
        times.append(dt)
        psteps.append(steps)
        if i in batched:
            b, bsteps, _ = batched[i]
            if bsteps != steps:
                rho = serving.solve_plain(p64, reqs[i], 0.0, check_every, bsteps)[0]
            diffs.append(float(np.max(np.abs(b.reshape(rho.shape) - rho)) / np.max(np.abs(rho))))
    # accuracy at equilibrium: requests the FP32 server converged, solved to
    # convergence by the plain FP64 path too, final states compared
    conv_ids = [i for i in sorted(batched) if batched[i][2] == F.FL_OK][:accuracy_subset]
    eq_diffs = []
    for i in conv_ids:
        rho, steps, res, conv, dt = serving.solve_plain(p64, reqs[i], tol, check_every, max_steps)
        if conv:
            b = batched[i][0]
            eq_diffs.append(float(np.max(np.abs(b.reshape(rho.shape) - rho)) / np.max(np.abs(rho))))
    plain_rate = len(idx) / sum(times)
    strip = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items() if k != "records"}
    return {
        "requests": len(reqs), "rejected_feed_draws": rejected, "tol": tol, "check_every": check_every,
        "max_steps": max_steps, "pool_MB": pool_mb, "tick_ms": tick_ms, "precision": "fp32 populations",
        "admission": policy,
        "closed_loop": strip(closed),
        "open_loop": dict(strip(opened), arrival_rate_per_s=round(rate, 3)),
        "plain_fp64": {"subset": len(idx), "solves_per_s": round(plain_rate, 3),
                       "p50_service_s": round(float(np.percentile(times, 50)), 4),
                       "p99_service_s": round(float(np.percentile(times, 99)), 4),
                       "mean_steps": float(np.mean(psteps))},
        "speedup_vs_plain_fp64": round(opened["solves_per_s"] / plain_rate, 2),
        "equilibrium_accuracy": {"requests": len(eq_diffs),
                                 "max_rel_diff_fp32_batched_vs_fp64_plain": max(eq_diffs) if eq_diffs else None},
        "equal_step_drift": {"requests": len(diffs),
                             "max_rel_diff_fp32_batched_vs_fp64_plain": max(diffs) if diffs else None},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="binary_slab_3d", choices=sorted(wl.WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched serving leg")
    ap.add_argument("--serve-policy", default="largest_first", choices=["largest_first", "fifo"],
                    help="order in which arrived requests are admitted")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-max-steps", type=int, default=50000)
    ap.add_argument("--serve-pool-mb", type=int, default=256, help="HBM budget of the server pool")
    ap.add_argument("--serve-tick-ms", type=float, default=50.0,
                    help="wall-clock budget of one batched-kernel tick")
    ap.add_argument("--state", default="workload", choices=["workload", "uniform"],
                    help="uniform: the workload's mean composition everywhere (a steady state; the "
                         "per-step work does not depend on the state)")
    ap.add_argument("--stencil", default="axis", choices=["axis", "isotropic"],
                    help="gradient and Laplacian stencils of the force (isotropic: the lattice-"
                         "weighted ones that keep 3-D droplets in the EOS domain)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="print the attainable HBM rates of the kernels' access patterns and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (PMC byte-counter scale)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the solver runs on one GPU (the multi-GPU decomposition is a design, not "
              "an implementation); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.stream_probe:
        import ctypes
        from paper_2212_10680_amd import build as B
        if not os.path.exists(B.PROBE_LIB):
            raise ImportError(f"{B.PROBE_LIB} is not built: run python -m paper_2212_10680_amd.build")
        lib = ctypes.CDLL(B.PROBE_LIB)
        buf = ctypes.create_string_buffer(1 << 14)
        rc = lib.flp_stream_probe(buf, len(buf))
        print(buf.value.decode(), end="")
        sys.exit(0 if rc == 0 else 1)
    F.load()  # fails loudly when the HIP library is not built

    w = wl.WORKLOADS[args.workload]
    precision = args.precision or w.precision
    p = F.Params.from_workload(w, precision=precision, stencil=args.stencil)
    solver = F.Solver(p)
    rho, u = wl.initial_field(w)
    if args.state == "uniform":
        rho = np.ascontiguousarray(np.broadcast_to(rho.reshape(w.ncomp, -1).mean(axis=1)[:, None],
                                                   (w.ncomp, w.nodes)))
        u = None
    solver.set_state(rho, u)
    print(f"[bench] {w.name} {w.lattice} {w.shape} nc={w.ncomp} {w.collision} tau={w.tau} {precision} "
          f"{args.stencil} stencils",
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
    solver.step_timed(0)  # creates the solver's timing events outside the timed region
    torch.cuda.synchronize()
    # the timed region: exactly K steps; HIP events on the solver's stream
    # around the kernels of every TIMING_EVERY-th step give the per-kernel
    # launch durations (events on every step would add ~10 us per step)
    t0 = time.perf_counter()
    kavg, timed_launches = solver.step_timed_every(args.steps, TIMING_EVERY)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {wall:.3f} s ({timed_launches} of them with events)",
          file=sys.stderr, flush=True)

    nodes = w.nodes
    ms_per_step = 1e3 * wall / args.steps
    value = nodes * w.ncomp * args.steps / wall / 1e6
    ab = algorithmic_bytes(w, precision)
    dominant = max(kavg, key=kavg.get)
    avg_ms = kavg[dominant]
    achieved = ab[dominant] * nodes / (avg_ms * 1e-3) / 1e9
    step_gpu_ms = sum(kavg.values())
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        # the stored counters were taken with the axis stencils
        "traffic": stored_traffic(dominant, nodes) if args.stencil == "axis" else None,
        "kernel": dominant,
        "kernel_avg_ms": round(avg_ms, 4),
        "algorithmic_bytes_per_node": ab[dominant],
        "kernel_ms_per_step": {k: round(v, 4) for k, v in kavg.items()},
        "timed_launches_per_kernel": timed_launches,
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
        "config": {"workload": w.name, "state": args.state, "stencil": args.stencil, "lattice": w.lattice,
                   "shape": list(w.shape),
                   "ncomp": w.ncomp,
                   "collision": w.collision, "tau": w.tau, "precision": precision,
                   "node_MLUPS": round(nodes * args.steps / wall / 1e6, 1)},
        "roofline": roofline,
        "mass_total": [float(m) for m in mass],
    }
    if not args.no_serving:
        out["serving"] = serving_bench(n_requests=args.serve_requests, max_steps=args.serve_max_steps,
                                       tick_ms=args.serve_tick_ms, pool_mb=args.serve_pool_mb,
                                       policy=args.serve_policy)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
