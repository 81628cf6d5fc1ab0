#!/usr/bin/env python3
"""Benchmark of the per-time-step update on one MI355X.

Default workload: D3Q19 256^3 periodic ternary lattice with two liquid
droplets (radius 30, centres 70 apart, approaching at +-0.02) in vapor, PR EOS,
MRT tau = 0.8, FP32 populations with FP64 EOS logarithms, and the isotropic
lattice stencils that keep 3-D droplets in the EOS domain (the largest
single-GPU configuration).  A step is one pass of the whole update (moments +
EOS, then forces + collision + streaming) over every node; inputs are resident
in HBM before the timed region.  The same lattice in the plain FP64 form and
the 128^3 binary slab (BGK tau = 0.8, the paper's axis stencils) are measured
after it and reported under "extra_configs".

Prints ONE JSON line: component-MLUPS of the whole job, the roofline of the
dominant kernel (algorithmic bytes per launch / average launch duration, HIP
events on the solver's stream), the batched-serving block, and the FP64 oracle
timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
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


def algorithmic_bytes(w, precision, stencil="axis", lap_pass=None):
    """Algorithmic HBM bytes per node of each kernel of one step.

    k_moments_eos: read every population, write rho~_i, ln f_i and phi (FP64).
    k_collide_stream / k_collide_zmarch (the same work; the second stages the
    FP64 fields through LDS): read and write every population, read rho~_i,
    ln f_i and phi (axis stencils) or -lap(phi) (isotropic stencils) once (the
    stencil re-reads are cache traffic), read and write the previous force sum
    (D values).  The FP32 form also reads the rest-population reference.
    k_interface_lap (isotropic stencils, when the collide pass is the
    one-thread-per-node kernel): read phi, write -lap(phi).
    k_collide_zmarch_iso (isotropic stencils, z-marching; with three components
    k_collide_zmarch_iso_cs, one thread group per component): reads phi instead
    of -lap(phi), which it forms itself; no Laplacian pass then runs.
    k_fused_step: the whole step, i.e. the per-node-step figure.
    """
    Q = 9 if w.lattice == "D2Q9" else 19
    D = w.D
    nc = w.ncomp
    s = 8 if precision == "fp64" else 4
    ref = 0 if precision == "fp64" else 4 * nc
    pops = Q * nc * s
    aux = 8 * (2 * nc + 1)          # rho~_i, ln f_i and phi or -lap(phi) (FP64)
    k1 = pops + ref + aux
    k2 = 2 * pops + ref + aux + 2 * s * D
    if lap_pass is None:
        lap_pass = stencil == "isotropic"
    lap = 16 if lap_pass else 0
    # per-node-step figure: populations once in and out, the FP64 densities,
    # ln f and the interface field once each way, the force history (population
    # precision) once each way, the FP32 form's rest-population reference once,
    # and with the isotropic stencils the Laplacian pass (phi in, -lap(phi) out)
    step = 2 * pops + 2 * aux + 2 * s * D + ref + lap
    out = {"k_moments_eos": k1, "k_collide_stream": k2, "k_collide_zmarch": k2, "k_collide_zmarch_iso": k2,
           "k_collide_zmarch_iso_cs": k2,
           "k_fused_step": step, "step": step}
    if lap:
        out["k_interface_lap"] = lap
    return out


def _row_precision(row):
    """Population precision of a traffic row: its own field, else read off the
    kernel's template arguments."""
    return row.get("precision") or ("fp64" if "double" in row.get("template", "") else "fp32")


def _row_key(row):
    return (row.get("kernel"), row.get("nodes"), row.get("stencil", "axis"), _row_precision(row))


def stored_traffic(kernel, nodes, stencil="axis", precision="fp32"):
    """HBM bytes per launch from the committed PMC counters, if they were taken
    on the current kernel sources for this kernel, lattice size, stencil and
    population precision (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    for k in t.get("kernels", []):
        if _row_key(k) == (kernel, nodes, stencil, precision):
            return k.get("bytes_per_launch")
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, stencil="axis", budget_s=12.0, single_budget_s=8.0):
    """FP64 oracle (as it stands) on a bounded slice of the workload, on all
    host threads and on one; an oracle failure is reported, not raised."""
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
    nodes = int(np.prod(shape))
    all_threads = lbm.num_threads()

    def rate(threads, budget):
        lbm.set_threads(threads)
        o = lbm.OracleLBM(mix, w.lattice, shape, tau=w.tau, collision=w.collision, stencil=stencil)
        o.init(rho.reshape(w.ncomp, -1), None if u is None else u.reshape(w.D, -1))
        o.run(1)  # warm-up
        steps = 0
        t0 = time.perf_counter()
        while True:
            o.run(1)
            steps += 1
            if time.perf_counter() - t0 > budget or steps >= 10000:
                break
        dt = time.perf_counter() - t0
        return nodes * w.ncomp * steps / dt / 1e6, steps, dt

    out = {"unit": "component-MLUPS", "kind": "oracle", "cpu_model": cpu_model(), "cores": all_threads}
    try:
        v, steps, dt = rate(all_threads, budget_s)
        v1, steps1, dt1 = rate(1, single_budget_s)
    except FloatingPointError as e:
        out.update({"value": None, "error": str(e)})
        return out
    finally:
        lbm.set_threads(all_threads)
    out.update({"value": round(v, 3), "single_thread_value": round(v1, 3),
                "sample": f"{w.lattice} {'x'.join(map(str, shape))} slice of the workload ({stencil} stencils), "
                          f"FP64, {w.collision}: {steps} steps in {dt:.1f} s on {all_threads} threads, "
                          f"{steps1} steps in {dt1:.1f} s on 1 thread"})
    return out


def serving_bench(n_requests=512, max_steps=50000, pool_mb=256, tick_ms=50.0, plain_subset=16,
                  tol=1e-10, check_every=1000, accuracy_subset=48, policy="largest_first", tuning=None):
    """Batched VLE serving: FP32-population server vs the plain FP64 path.

    Requests: binary D2Q9 L x 8 slabs, L log-uniform in [64, 2048], feed z1
    redrawn until a S_V = 0.5 state exists; each runs until the rate residual is
    below tol (checked every check_every steps) or max_steps.  Closed loop first
    (all requests present at t = 0), then a seeded Poisson stream at 0.8 of the
    closed loop's completion rate, admitted by the pool budget.  Throughput and
    time to equilibrium count converged requests only.  The relaxation time of a
    slab grows like a power of L, so max_steps caps the larger lattices: the
    fitted law and the largest L it lets converge are reported with the cap.
    Accuracy and the comparison with the plain FP64 path use the requests the
    FP32 server converged: the same requests solved to convergence in FP64.
    """
    from paper_2212_10680_amd import serving

    w = wl.WORKLOADS["serving_binary_2d"]
    p32 = F.Params.from_workload(w, precision="fp32")
    p64 = F.Params.from_workload(w, precision="fp64")
    reqs, rejected = wl.serving_requests(n=n_requests, seed=0)
    srv = F.Server(p32, pool_bytes=pool_mb << 20, max_slots=512)
    srv.set_tuning(tuning)
    closed = serving.serve(srv, reqs, np.zeros(len(reqs)), tol, check_every, max_steps, tick_ms, policy=policy)
    srv.close()
    print(f"[bench] serving closed loop: {closed['converged']} of {closed['requests']} converged, "
          f"{closed['converged_solves_per_s']:.1f} converged solves/s", file=sys.stderr, flush=True)
    recs = closed["records"]
    span = max(r["done"] for r in recs)
    rate = 0.8 * len(recs) / span
    arrivals = serving.poisson_arrivals(len(reqs), rate, seed=0)
    srv = F.Server(p32, pool_bytes=pool_mb << 20, max_slots=512)
    srv.set_tuning(tuning)
    batched = {}
    opened = serving.serve(srv, reqs, arrivals, tol, check_every, max_steps, tick_ms, policy=policy,
                           on_result=lambda rec, rho: batched.__setitem__(rec["i"], (rho, rec["steps"], rec["status"])))
    srv.close()
    print(f"[bench] serving open loop: {opened['converged_solves_per_s']:.1f} converged solves/s, "
          f"p99 time to equilibrium {opened['p99_time_to_equilibrium_s']:.2f} s", file=sys.stderr, flush=True)

    # relaxation law of the converged requests: steps ~ a L^alpha
    conv = [r for r in recs if r["status"] == F.FL_OK]
    fit = None
    if len(conv) >= 4 and len({r["L"] for r in conv}) >= 2:
        Ls = np.array([r["L"] for r in conv], float)
        st = np.array([r["steps"] for r in conv], float)
        alpha, loga = np.polyfit(np.log(Ls), np.log(st), 1)
        fit = {"alpha": round(float(alpha), 3), "a": float(np.exp(loga)),
               "largest_L_within_cap": round(float((max_steps / np.exp(loga)) ** (1.0 / alpha)), 1),
               "steps_needed_at_L_2048": float(np.exp(loga) * 2048.0 ** alpha)}

    # the converged set C: accuracy against FP64 and the plain-path comparison
    conv_ids = sorted(i for i in batched if batched[i][2] == F.FL_OK)
    acc_ids = conv_ids[:: max(1, len(conv_ids) // accuracy_subset)][:accuracy_subset]
    acc = {}
    if acc_ids:
        # the FP64 server is bitwise equal to the plain FP64 single-lattice path
        # (tests/test_gpu_serving.py); it solves the subset in one batch
        sub = [reqs[i] for i in acc_ids]
        srv = F.Server(p64, pool_bytes=pool_mb << 20, max_slots=512)
        srv.set_tuning(tuning)
        ref = serving.serve(srv, sub, np.zeros(len(sub)), tol, check_every, 4 * max_steps, tick_ms,
                            on_result=lambda rec, rho: acc.__setitem__(acc_ids[rec["i"]], (rho, rec["status"])))
        srv.close()
    diffs, Lacc = [], []
    for i in acc_ids:
        if i in acc and acc[i][1] == F.FL_OK:
            rho = acc[i][0]
            b = batched[i][0]
            diffs.append(float(np.max(np.abs(b.reshape(rho.shape) - rho)) / np.max(np.abs(rho))))
            Lacc.append(reqs[i]["L"])
    # throughput on equal work: the converged set C on the batched FP32 server
    # (all admitted at once) and a spread subset of C on the plain FP64 path
    # (one request at a time, two kernels per step)
    sub = [reqs[i] for i in conv_ids]
    srv = F.Server(p32, pool_bytes=pool_mb << 20, max_slots=512)
    srv.set_tuning(tuning)
    cset = serving.serve(srv, sub, np.zeros(len(sub)), tol, check_every, max_steps, tick_ms, policy=policy)
    srv.close()
    idx = conv_ids[:: max(1, len(conv_ids) // plain_subset)][:plain_subset]
    times, psteps, pconv = [], [], 0
    for i in idx:
        rho, steps, res, ok, dt = serving.solve_plain(p64, reqs[i], tol, check_every, 4 * max_steps)
        times.append(dt)
        psteps.append(steps)
        pconv += bool(ok)
    plain_rate = len(idx) / sum(times) if times else None
    strip = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items() if k != "records"}
    return {
        "requests": len(reqs), "rejected_feed_draws": rejected, "tol": tol, "check_every": check_every,
        "max_steps": max_steps, "pool_MB": pool_mb, "tick_ms": tick_ms, "precision": "fp32 populations",
        "admission": policy,
        "closed_loop": strip(closed),
        "open_loop": dict(strip(opened), arrival_rate_per_s=round(rate, 3)),
        "cap": {"relaxation_fit_steps_vs_L": fit,
                "note": "steps to a rate residual below tol grow like a power of L; requests whose "
                        "relaxation needs more than max_steps stop there (status FL_ENOTCONV) and are "
                        "not counted as solves"},
        "converged_set": {"requests": len(conv_ids), "batched_fp32": strip(cset),
                          "plain_fp64": {"subset": len(idx), "converged": pconv,
                                         "solves_per_s": round(plain_rate, 3) if plain_rate else None,
                                         "p50_service_s": round(float(np.percentile(times, 50)), 4) if times else None,
                                         "p99_service_s": round(float(np.percentile(times, 99)), 4) if times else None,
                                         "mean_steps": float(np.mean(psteps)) if psteps else None},
                          "speedup_batched_fp32_vs_plain_fp64":
                              round(cset["converged_solves_per_s"] / plain_rate, 2) if plain_rate else None},
        "equilibrium_accuracy": {"requests": len(diffs), "L_range": [min(Lacc), max(Lacc)] if Lacc else None,
                                 "max_rel_diff_fp32_batched_vs_fp64": max(diffs) if diffs else None},
    }


def _kernel_short(name):
    """'void fl::k_collide_stream<1, 3, float, true, true>(...)' -> 'k_collide_stream'."""
    m = re.search(r"fl::(k_[a-z0-9_]+)", name)
    return m.group(1) if m else name.split("(")[0]


def _pmc_per_dispatch(csv_path):
    """{kernel name: [counter value per dispatch]} of a rocprofv3 --pmc CSV
    (one counter; rows repeated for one dispatch are counted once)."""
    seen, out = set(), {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            key = (row["Dispatch_Id"], row["Counter_Name"])
            if key in seen:
                continue
            seen.add(key)
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def write_traffic(fetch_csv, write_csv, w, stencil, copy_bytes=1 << 30):
    """HBM bytes per launch of each kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
    `bench.py --copy-calibration`: each counter is scaled by what it reads for
    the 1 GiB device copy in the same run (copy_bytes read and written).
    Updates profiles/traffic.json (a row per kernel, lattice size, stencil and
    population precision; rows taken on other kernel sources are dropped) and
    prints a markdown table of this run's rows."""
    fetch, write = _pmc_per_dispatch(fetch_csv), _pmc_per_dispatch(write_csv)

    def scale(d):
        vals = [v for k, vs in d.items() if "copyBuffer" in k or "copy" in k.lower() for v in vs
                if v * 1024 > 0.25 * copy_bytes]
        if not vals:
            raise SystemExit("no 1 GiB copy dispatch in the counter file (run with --copy-calibration)")
        return copy_bytes / (1024.0 * float(np.mean(vals)))

    sf, sw = scale(fetch), scale(write)
    rows = []
    for name in sorted(set(fetch) & set(write)):
        if "fl::" not in name:
            continue
        r = float(np.mean(fetch[name])) * 1024 * sf
        wbytes = float(np.mean(write[name])) * 1024 * sw
        row = {"kernel": _kernel_short(name), "template": name.split("(")[0].replace("void ", ""),
               "workload": w.name, "nodes": w.nodes, "stencil": stencil, "launches": len(fetch[name]),
               "read_bytes": round(r), "write_bytes": round(wbytes), "bytes_per_launch": round(r + wbytes),
               "bytes_per_node": round((r + wbytes) / w.nodes, 1)}
        row["precision"] = _row_precision(row)
        row["scale"] = {"FETCH_SIZE": sf, "WRITE_SIZE": sw}
        rows.append(row)
    # rows of other kernels, sizes, stencils or precisions taken on the same
    # kernel sources are kept; rows from other sources are dropped
    kept = []
    try:
        with open(TRAFFIC_FILE) as f:
            old = json.load(f)
        if old.get("kernel_source_hash") == kernel_source_hash():
            new_keys = {_row_key(r) for r in rows}
            kept = [r for r in old.get("kernels", []) if _row_key(r) not in new_keys]
            for r in kept:
                r.setdefault("precision", _row_precision(r))
                r.setdefault("scale", old.get("scale"))
    except (OSError, ValueError):
        pass
    out = {"kernel_source_hash": kernel_source_hash(), "date": time.strftime("%Y-%m-%d"),
           "scale": {"FETCH_SIZE": sf, "WRITE_SIZE": sw}, "kernels": kept + rows}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(f"Scale factors from a {copy_bytes >> 20} MiB device copy: FETCH_SIZE x{sf:.4f}, WRITE_SIZE x{sw:.4f}.\n")
    print("| kernel | launches | scaled read MB | scaled write MB | bytes/node |")
    print("|---|---|---|---|---|")
    for r in rows:
        print(f"| `{r['template']}` | {r['launches']} | {r['read_bytes'] / 1e6:.1f} | {r['write_bytes'] / 1e6:.1f} | "
              f"{r['bytes_per_node']} |")


def trace_summary(stats_csv):
    """Markdown table of a rocprofv3 --kernel-trace --stats kernel_stats.csv."""
    print("| kernel | calls | avg us | min us | max us | % time |")
    print("|---|---|---|---|---|---|")
    with open(stats_csv) as f:
        for row in csv.DictReader(f):
            name = row["Name"].split("(")[0].replace("void ", "")
            print(f"| `{name}` | {row['Calls']} | {float(row['AverageNs']) / 1e3:.1f} | "
                  f"{float(row['MinNs']) / 1e3:.1f} | {float(row['MaxNs']) / 1e3:.1f} | "
                  f"{float(row['Percentage']):.2f} |")


def default_stencil(w):
    """The isotropic stencils for droplets in 3-D (the axis ones leave the EOS
    domain there within tens of steps), the paper's axis stencils otherwise."""
    return "isotropic" if (w.D == 3 and w.geometry in ("droplet", "two_droplets")) else "axis"


def measure_lattice(w, precision, stencil, state, steps, warmup, tuning=None):
    """Time exactly `steps` steps of one lattice after `warmup` untimed ones;
    returns the throughput, the per-kernel launch times and the roofline."""
    import torch

    p = F.Params.from_workload(w, precision=precision, stencil=stencil)
    solver = F.Solver(p)
    if tuning:
        solver.set_tuning(tuning)
    rho, u = wl.initial_field(w)
    if state == "uniform":
        rho = np.ascontiguousarray(np.broadcast_to(rho.reshape(w.ncomp, -1).mean(axis=1)[:, None],
                                                   (w.ncomp, w.nodes)))
        u = None
    solver.set_state(rho, u)
    del rho, u
    print(f"[bench] {w.name} {w.lattice} {w.shape} nc={w.ncomp} {w.collision} tau={w.tau} {precision} "
          f"{stencil} stencils", file=sys.stderr, flush=True)
    solver.step(warmup)
    torch.cuda.synchronize()
    tw = time.perf_counter()
    solver.step(2)  # two more untimed steps: how long a step takes (first launches are behind)
    torch.cuda.synchronize()
    warm_ms = (time.perf_counter() - tw) * 1e3 / 2
    solver.step_timed(0)  # creates the solver's timing events outside the timed region
    torch.cuda.synchronize()
    # the timed region: exactly K steps; HIP events on the solver's stream
    # around the kernels give the per-kernel launch durations: on every step
    # when a step takes a millisecond or more (the events add ~10 us per
    # step), else on every TIMING_EVERY-th one
    every = 1 if warm_ms >= 1.0 else TIMING_EVERY
    t0 = time.perf_counter()
    kavg, timed_launches = solver.step_timed_every(steps, every)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] timed {steps} steps in {wall:.3f} s ({timed_launches} of them with events)",
          file=sys.stderr, flush=True)
    nodes = w.nodes
    ab = algorithmic_bytes(w, precision, stencil, lap_pass="k_interface_lap" in kavg)
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
        "traffic": stored_traffic(dominant, nodes, stencil, precision),
        "kernel": dominant,
        "kernel_avg_ms": round(avg_ms, 4),
        "algorithmic_bytes_per_node": ab[dominant],
        "kernel_ms_per_step": {k: round(v, 4) for k, v in kavg.items()},
        "kernel_frac": {k: round(ab[k] * nodes / (v * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4) for k, v in kavg.items()},
        "timed_launches_per_kernel": timed_launches,
        "step_effective_GBps": round(ab["step"] * nodes / (step_gpu_ms * 1e-3) / 1e9, 1),
        "step_effective_frac": round(ab["step"] * nodes / (step_gpu_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "step_bytes_per_node": ab["step"],
    }
    mass = solver.mass()
    solver.close()
    del solver
    torch.cuda.empty_cache()
    return {
        "value": round(nodes * w.ncomp * steps / wall / 1e6, 1),
        "ms_per_step": round(1e3 * wall / steps, 4),
        "steps": steps,
        "warmup": warmup,
        "config": {"workload": w.name, "state": state, "stencil": stencil, "lattice": w.lattice,
                   "shape": list(w.shape), "ncomp": w.ncomp, "collision": w.collision, "tau": w.tau,
                   "precision": precision, "node_MLUPS": round(nodes * steps / wall / 1e6, 1)},
        "roofline": roofline,
        "mass_total": [float(m) for m in mass],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ternary_droplets_3d", choices=sorted(wl.WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched serving leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the FP64 form and the 128^3 binary slab after the headline")
    ap.add_argument("--serve-policy", default="largest_first", choices=["largest_first", "fifo"],
                    help="order in which arrived requests are admitted")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-tuning", default=None, help="launch tuning spec passed to fl_server_set_tuning")
    ap.add_argument("--serve-max-steps", type=int, default=50000)
    ap.add_argument("--serve-pool-mb", type=int, default=256, help="HBM budget of the server pool")
    ap.add_argument("--serve-tick-ms", type=float, default=50.0,
                    help="wall-clock budget of one batched-kernel tick")
    ap.add_argument("--state", default="workload", choices=["workload", "uniform"],
                    help="uniform: the workload's mean composition everywhere (a steady state; the "
                         "per-step work does not depend on the state)")
    ap.add_argument("--stencil", default=None, choices=["axis", "isotropic"],
                    help="gradient and Laplacian stencils of the force (default: isotropic for 3-D "
                         "droplets, which leave the EOS domain with the axis ones; axis otherwise)")
    ap.add_argument("--tuning", default=None, help="launch tuning spec passed to fl_set_tuning")
    ap.add_argument("--stream-probe", action="store_true",
                    help="print the attainable HBM rates of the kernels' access patterns and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (PMC byte-counter scale)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter files of a "
                         "--copy-calibration run (no GPU needed) and exit")
    ap.add_argument("--trace-summary", metavar="KERNEL_STATS_CSV",
                    help="print a markdown table of a rocprofv3 --stats kernel_stats.csv and exit")
    args = ap.parse_args()

    if args.traffic_from or args.trace_summary:
        w = wl.WORKLOADS[args.workload]
        if args.traffic_from:
            write_traffic(*args.traffic_from, w, args.stencil or default_stencil(w))
        else:
            trace_summary(args.trace_summary)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the solver runs on one GPU (cutting the lattice into z-slabs over "
              "several GPUs is designed, not implemented); use --gpus 1", file=sys.stderr)
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
        if rc == 0:
            buf = ctypes.create_string_buffer(1 << 14)
            rc = lib.flp_zmarch_probe(buf, len(buf))
            print(buf.value.decode(), end="")
        sys.exit(0 if rc == 0 else 1)
    F.load()  # fails loudly when the HIP library is not built

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
        torch.cuda.empty_cache()

    w = wl.WORKLOADS[args.workload]
    precision = args.precision or w.precision
    stencil = args.stencil or default_stencil(w)
    head = measure_lattice(w, precision, stencil, args.state, args.steps, args.warmup, args.tuning)
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "component-MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 populations / f64 EOS" if precision == "fp32" else "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "mass_total": head["mass_total"],
    }
    if not args.no_extra:
        extra = {}
        # the other lattices are timed over at least 200 steps: the fixed cost
        # around a timed region (about 0.5 ms of synchronisation) would
        # otherwise weigh 10 % on the 0.22 ms step of the 128^3 slab at 20 steps
        xs, xw = max(args.steps, 200), max(args.warmup, 20)
        if precision != "fp64":
            # the plain FP64 form of the same lattice (both forms are reported)
            extra[f"{w.name}_fp64"] = measure_lattice(w, "fp64", stencil, args.state, xs, xw, args.tuning)
        if args.workload != "binary_slab_3d":
            wx = wl.WORKLOADS["binary_slab_3d"]
            extra["binary_slab_3d"] = measure_lattice(wx, wx.precision, "axis", "workload", xs, xw)
        out["extra_configs"] = extra
    if not args.no_serving:
        out["serving"] = serving_bench(n_requests=args.serve_requests, max_steps=args.serve_max_steps,
                                       tick_ms=args.serve_tick_ms, pool_mb=args.serve_pool_mb,
                                       policy=args.serve_policy,
                                       tuning=args.serve_tuning)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, stencil=stencil)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
