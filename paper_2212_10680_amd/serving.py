"""Request loop of the batched VLE server.

Requests arrive as a seeded Poisson stream; a request is admitted when a
server slot and enough pool memory are free (admission by HBM budget); every
tick advances all admitted, unfinished requests in one batched kernel launch;
finished requests are collected and their latency (arrival to collection)
recorded.  The plain comparison path solves the same requests one after
another with the single-lattice solver.
"""
from __future__ import annotations

import heapq
import time
from collections import deque

import numpy as np

from . import fuglbm as F
from . import workloads as wl


def request_field(req, W=4.0, SV=0.5):
    """Initial molar densities of one request (tanh slab, eq. eqInit)."""
    L, ny = req["L"], req["ny"]
    x = np.arange(L, dtype=np.float64)
    prof = np.stack([wl.slab_profile(x, L, req["rho_L"][i], req["rho_V"][i], SV, W)
                     for i in range(len(req["rho_L"]))])
    return np.ascontiguousarray(np.repeat(prof[:, None, :], ny, axis=1))


def poisson_arrivals(n, rate, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / rate, n))


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def serve(server: F.Server, reqs, arrivals, tol, check_every, max_steps, tick_ms=20.0,
          time_limit_s=None, on_result=None, policy="largest_first"):
    """Run the request stream through the server.  Wall-clock times in seconds
    from the start; arrivals[i] is request i's arrival time.  policy is the
    order in which arrived, not yet admitted requests are offered to the
    server: "largest_first" (the longest lattices first: each runs on one
    workgroup, so the last long solve to start sets the makespan) or "fifo"."""
    if policy not in ("largest_first", "fifo"):
        raise ValueError(f"unknown admission policy {policy!r}")
    order = np.argsort(arrivals, kind="stable")
    pending = deque(int(i) for i in order)
    waiting = []  # heap of arrived requests: (priority, arrival rank, index)
    rank = 0
    inflight = {}
    admitted = {}
    done = []
    t0 = time.perf_counter()
    ticks = 0
    rejected_admissions = 0
    while pending or waiting or inflight:
        now = time.perf_counter() - t0
        while pending and arrivals[pending[0]] <= now:
            i = pending.popleft()
            prio = -reqs[i]["L"] * reqs[i]["ny"] if policy == "largest_first" else 0
            heapq.heappush(waiting, (prio, rank, i))
            rank += 1
        while waiting:
            i = waiting[0][2]
            r = reqs[i]
            rid = server.submit(request_field(r), (r["L"], r["ny"]), tol, check_every, max_steps)
            if rid is None:
                rejected_admissions += 1
                break
            heapq.heappop(waiting)
            inflight[rid] = i
            admitted[i] = time.perf_counter() - t0
        if not inflight:
            if waiting:
                raise RuntimeError("a request cannot be admitted into an empty server")
            if pending:
                wait = arrivals[pending[0]] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
            continue
        server.tick(max_steps, tick_ms)
        ticks += 1
        for rid in server.poll():
            i = inflight.pop(rid)
            r = reqs[i]
            out = server.result(rid, r["L"] * r["ny"], full=True)
            t = time.perf_counter() - t0
            rec = {"i": i, "L": r["L"], "steps": out["steps"], "residual": out["residual"],
                   "status": out["status"], "arrival": float(arrivals[i]), "admitted": admitted[i], "done": t,
                   "latency": t - float(arrivals[i]), "service_s": out["latency_s"]}
            done.append(rec)
            if on_result:
                on_result(rec, out["rho_molar"])
        if time_limit_s and time.perf_counter() - t0 > time_limit_s:
            break
    wall = time.perf_counter() - t0
    conv = [d for d in done if d["status"] == F.FL_OK]
    lat = [d["latency"] for d in conv]
    span = (max(d["done"] for d in done) - min(d["arrival"] for d in done)) if done else float("nan")
    return {
        "requests": len(reqs), "completed": len(done),
        "converged": len(conv),
        "max_steps_reached": sum(d["status"] == F.FL_ENOTCONV for d in done),
        "numeric_failures": sum(d["status"] == F.FL_ENUMERIC for d in done),
        # throughput and latency count converged requests only (arrival to the
        # result of a request whose residual fell below tol); requests stopped at
        # max_steps or by a numeric failure are reported above, not counted here
        "converged_solves_per_s": len(conv) / span if conv else 0.0,
        "p50_time_to_equilibrium_s": percentile(lat, 50), "p99_time_to_equilibrium_s": percentile(lat, 99),
        "largest_converged_L": max((d["L"] for d in conv), default=None),
        "wall_s": wall, "ticks": ticks, "admission_waits": rejected_admissions,
        "records": done,
    }


def solve_plain(params: F.Params, req, tol, check_every, max_steps, precision="fp64"):
    """One request with the single-lattice solver (two kernels per step)."""
    s = F.Solver(params.with_shape((req["L"], req["ny"]), precision=precision))
    s.set_state(request_field(req))
    t = time.perf_counter()
    conv, steps, res = s.run_until(tol, check_every, max_steps)
    dt = time.perf_counter() - t
    rho = s.fields()["rho_molar"]
    s.close()
    return rho, steps, res, conv, dt
