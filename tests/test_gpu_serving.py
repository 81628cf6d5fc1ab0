"""Batched server (fl_server_*) on the GPU, through the C ABI.

* each request's result equals the single-lattice solver's (same kernels' node
  arithmetic, same residual checks) bitwise;
* a request's result is bitwise the same alone and in a mix, whatever the tick
  size (continuous batching does not change per-request arithmetic);
* admission is bounded by the pool budget and the slot count;
* a request that leaves the EOS domain fails alone;
* the FP32-population server agrees with the FP64 oracle within 1e-4.
"""
import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import serving
from paper_2212_10680_amd import workloads as wl

from _util import oracle_for, rel

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def base_params(precision="fp32"):
    return F.Params.from_workload(wl.WORKLOADS["serving_binary_2d"], precision=precision)


def some_requests(n, seed=0):
    reqs, _ = wl.serving_requests(n=n, seed=seed, L_min=32, L_max=160)
    return reqs


def run_server(p, reqs, tol, check, max_steps, tick, pool=1 << 28, order=None, tune=None):
    srv = F.Server(p, pool_bytes=pool, max_slots=64)
    srv.set_tuning(tune)
    ids = {}
    for i in (order if order is not None else range(len(reqs))):
        r = reqs[i]
        rid = srv.submit(serving.request_field(r), (r["L"], r["ny"]), tol, check, max_steps)
        assert rid is not None
        ids[rid] = i
    out = {}
    while len(out) < len(reqs):
        srv.tick(tick)
        for rid in srv.poll():
            i = ids[rid]
            out[i] = srv.result(rid, reqs[i]["L"] * reqs[i]["ny"])
    srv.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_server_equals_plain_solver_bitwise(precision):
    announce(f"server vs plain solver ({precision})")
    p = base_params(precision)
    reqs = some_requests(3)
    got = run_server(p, reqs, tol=0.0, check=250, max_steps=1500, tick=400)
    for i, r in enumerate(reqs):
        rho, steps, res, status = got[i]
        assert steps == 1500 and status == F.FL_ENOTCONV
        rho_p, steps_p, res_p, conv, _ = serving.solve_plain(p, r, 0.0, 250, 1500, precision=precision)
        assert steps_p == 1500 and not conv
        assert np.array_equal(rho, rho_p.reshape(rho.shape)), i
        assert res == res_p


def test_alone_vs_mix_bitwise():
    announce("alone vs mix")
    p = base_params("fp32")
    reqs = some_requests(6, seed=3)
    alone = run_server(p, reqs[:1], tol=1e-9, check=200, max_steps=3000, tick=3000)
    mix = run_server(p, reqs, tol=1e-9, check=200, max_steps=3000, tick=137, order=[3, 1, 0, 5, 2, 4])
    a, m = alone[0], mix[0]
    assert a[1] == m[1] and a[3] == m[3] and a[2] == m[2]
    assert np.array_equal(a[0], m[0])


def test_admission_by_pool_budget():
    announce("admission budget")
    p = base_params("fp32")
    req = dict(some_requests(1)[0], L=128)
    srv = F.Server(p, pool_bytes=1 << 20, max_slots=8)
    need = srv.request_bytes((128, 8))
    total = srv.info()["pool_total"]
    fits = total // need
    assert 1 <= fits < 8
    ids = []
    while True:
        rid = srv.submit(serving.request_field(req), (128, 8), 0.0, 100, 200)
        if rid is None:
            break
        ids.append(rid)
        assert len(ids) <= fits
    assert len(ids) == fits
    info = srv.info()
    assert info["pool_used"] == fits * need and info["active"] == fits
    srv.tick(500)
    assert srv.poll() and len(srv.poll()) == fits
    srv.result(ids[0], 128 * 8)
    assert srv.submit(serving.request_field(req), (128, 8), 0.0, 100, 200) is not None
    srv.close()


def test_slot_limit():
    announce("slot limit")
    p = base_params("fp32")
    req = some_requests(1)[0]
    srv = F.Server(p, pool_bytes=1 << 26, max_slots=2)
    f = serving.request_field(req)
    assert srv.submit(f, (req["L"], 8), 0.0, 100, 100) is not None
    assert srv.submit(f, (req["L"], 8), 0.0, 100, 100) is not None
    assert srv.submit(f, (req["L"], 8), 0.0, 100, 100) is None
    srv.close()


def test_failure_isolation():
    """A request driven out of the EOS domain fails alone; others are unaffected."""
    announce("failure isolation")
    p = base_params("fp32")
    reqs = some_requests(3, seed=5)
    good = run_server(p, reqs, tol=0.0, check=100, max_steps=600, tick=600)
    srv = F.Server(p, pool_bytes=1 << 26, max_slots=8)
    ids = {}
    for i, r in enumerate(reqs):
        ids[srv.submit(serving.request_field(r), (r["L"], 8), 0.0, 100, 600)] = i
    rng = np.random.default_rng(0)
    # in the EOS domain (rho~ b_m <= 0.90) but far from any stable state: the
    # FP64 oracle leaves the domain at its second step
    bad = np.stack([np.full((8, 32), 1.0), np.full((8, 32), 8.0)]) * (1 + 0.05 * rng.uniform(-1, 1, (2, 8, 32)))
    bad_id = srv.submit(bad, (32, 8), 0.0, 100, 600)
    assert bad_id is not None
    res = {}
    while len(res) < 4:
        srv.tick(600)
        for rid in srv.poll():
            n = 32 * 8 if rid == bad_id else reqs[ids[rid]]["L"] * 8
            res[rid] = srv.result(rid, n)
    assert res[bad_id][3] == F.FL_ENUMERIC
    for rid, i in ids.items():
        assert np.array_equal(res[rid][0], good[i][0])
    srv.close()


def test_server_fp32_vs_oracle():
    announce("server fp32 vs fp64 oracle")
    p = base_params("fp32")
    r = dict(some_requests(1, seed=2)[0], L=96)
    out = run_server(p, [r], tol=0.0, check=500, max_steps=2000, tick=2000)
    rho = out[0][0]
    w = wl.WORKLOADS["serving_binary_2d"].scaled((96, 8))
    o = oracle_for(w)
    o.init(serving.request_field(r).reshape(2, -1))
    o.run(2000)
    err = rel(rho.reshape(2, -1), o.fields()["rho_molar"])
    print(f"  rel diff {err:.2e}", flush=True)
    assert err < 1e-4


def test_convergence_status():
    announce("converges")
    p = base_params("fp32")
    r = dict(some_requests(1, seed=4)[0], L=32, ny=2)
    out = run_server(p, [r], tol=1e-8, check=500, max_steps=200000, tick=5000)
    rho, steps, res, status = out[0]
    print(f"  steps {steps} residual {res:.2e}", flush=True)
    assert status == F.FL_OK and res < 1e-8 and steps % 500 == 0


def test_request_cap_per_tick_bitwise():
    """Advancing at most two requests per tick (oldest first; the rest wait
    admitted) gives every request the same result, bit for bit, as advancing
    all of them, and every request completes."""
    announce("request cap per tick")
    reqs = some_requests(5, seed=7)
    capped = run_server(base_params("fp32"), reqs, tol=1e-9, check=200, max_steps=2000, tick=300,
                        tune="serve_cap=2")
    free = run_server(base_params("fp32"), reqs, tol=1e-9, check=200, max_steps=2000, tick=300,
                      tune="serve_cap=0")
    assert sorted(capped) == sorted(free) == list(range(len(reqs)))
    for i in range(len(reqs)):
        a, b = capped[i], free[i]
        assert a[1] == b[1] and a[2] == b[2] and a[3] == b[3], i
        assert np.array_equal(a[0], b[0]), i


def run_server_ms(p, reqs, tol, check, max_steps, tick, max_ms, tune):
    """run_server with time-sliced ticks (tick steps or max_ms of device time)."""
    srv = F.Server(p, pool_bytes=1 << 28, max_slots=64)
    srv.set_tuning(tune)
    ids = {}
    for i, r in enumerate(reqs):
        rid = srv.submit(serving.request_field(r), (r["L"], r["ny"]), tol, check, max_steps)
        assert rid is not None
        ids[rid] = i
    out = {}
    while len(out) < len(reqs):
        srv.tick(tick, max_ms)
        for rid in srv.poll():
            i = ids[rid]
            out[i] = srv.result(rid, reqs[i]["L"] * reqs[i]["ny"])
    srv.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_workgroup_groups_bitwise(precision):
    """Requests split over several workgroups of one XCD (serve_group: nodes
    per workgroup; groups of up to 8 that meet at a barrier twice per step)
    give the same result bit for bit as one workgroup per request: ten
    requests of 256 to 1 280 nodes at serve_group = 128 (groups of 2 to 8),
    with residual checks, converged and capped requests, and both with whole
    ticks and with ticks cut by a device-time budget."""
    announce(f"workgroup groups vs one workgroup per request ({precision})")
    p = base_params(precision)
    reqs = some_requests(10, seed=3)
    ref = run_server(p, reqs, tol=3e-6, check=100, max_steps=3000, tick=700, tune="serve_group=0")
    got = run_server(p, reqs, tol=3e-6, check=100, max_steps=3000, tick=700, tune="serve_group=128")
    sliced = run_server_ms(p, reqs, tol=3e-6, check=100, max_steps=3000, tick=5000, max_ms=0.3,
                           tune="serve_group=128")
    statuses = set()
    for i in range(len(reqs)):
        statuses.add(ref[i][3])
        for g in (got[i], sliced[i]):
            assert np.array_equal(ref[i][0], g[0]), i
            assert ref[i][1:] == g[1:], (i, ref[i][1:], g[1:])
    print(f"  statuses {sorted(statuses)}, steps {[ref[i][1] for i in range(len(reqs))]}", flush=True)


def test_workgroup_groups_fill_and_wait():
    """Grouped workgroups filling the device: 48 requests of 2 048 nodes in
    groups of 8 (a tick places groups while an XCD has room for one, at most
    the workgroups the device holds at once, the rest wait for later ticks);
    results bitwise equal to one workgroup per request."""
    announce("workgroup groups filling the device")
    p = base_params("fp32")
    reqs = [dict(r, L=256) for r in some_requests(48, seed=5)]
    ref = run_server(p, reqs, tol=0.0, check=200, max_steps=600, tick=250, tune="serve_group=0")
    got = run_server(p, reqs, tol=0.0, check=200, max_steps=600, tick=250, tune="serve_group=256")
    for i in range(len(reqs)):
        assert np.array_equal(ref[i][0], got[i][0]), i
        assert ref[i][1:] == got[i][1:], i
