"""fl_server_result_noalloc against fl_server_result, through the C ABI.

The no-alloc entry point stages a finished request's velocity and pressure in
a static device array instead of memory it allocates; its outputs must equal
the allocating entry point's bit for bit (the same kernel computes them), on
two calls in a row where the second request is smaller than the first (the
array keeps the first call's contents beyond the second request's size), and
a request larger than the array is rejected with FL_EINVAL.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import serving
from paper_2212_10680_amd import workloads as wl

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _collect(srv, rid, n, noalloc):
    lib = srv.lib
    p = srv.p
    rho = np.zeros((p.ncomp, n))
    u = np.zeros((p.D, n))
    pr = np.zeros(n)
    steps, res, st, lat = C.c_long(0), C.c_double(0.0), C.c_int(0), C.c_double(0.0)
    fn = lib.fl_server_result_noalloc if noalloc else lib.fl_server_result
    rc = fn(srv.h, C.c_uint64(rid), F._dp(rho), F._dp(u), F._dp(pr), C.byref(steps), C.byref(res), C.byref(st),
            C.byref(lat))
    return rc, rho, u, pr, steps.value, res.value, st.value


def test_noalloc_result_equals_allocating_result():
    announce("fl_server_result_noalloc vs fl_server_result")
    p = F.Params.from_workload(wl.WORKLOADS["serving_binary_2d"], precision="fp32")
    reqs, _ = wl.serving_requests(n=2, seed=5, L_min=64, L_max=400)
    big = dict(reqs[0], L=400)
    small = dict(reqs[1], L=72)
    srv = F.Server(p, pool_bytes=1 << 27, max_slots=8)
    ids = []
    for r in (big, big, small, small):
        rid = srv.submit(serving.request_field(r), (r["L"], r["ny"]), 0.0, 100, 300)
        assert rid is not None
        ids.append((rid, r["L"] * r["ny"]))
    while srv.tick(300) > 0:
        pass
    # two calls in a row on the static array: the larger request first, then
    # the smaller one; each against the allocating entry point on an identical
    # request (same initial field, same steps)
    for k in (0, 2):
        (ra, n), (rb, _) = ids[k], ids[k + 1]
        a = _collect(srv, ra, n, noalloc=False)
        b = _collect(srv, rb, n, noalloc=True)
        assert a[0] == F.FL_OK and b[0] == F.FL_OK
        for x, y in zip(a[1:4], b[1:4]):
            assert np.array_equal(x, y)
        assert a[4:] == b[4:] and a[4] == 300
        assert np.max(np.abs(b[2])) > 0.0 and np.all(b[3] > 0)
    # a request whose staging exceeds the array is refused, and stays collectable
    huge = dict(big, L=16384, ny=8)
    rid = srv.submit(serving.request_field(huge), (huge["L"], huge["ny"]), 0.0, 10, 10)
    assert rid is not None
    while srv.tick(10) > 0:
        pass
    n = huge["L"] * huge["ny"]
    rc = _collect(srv, rid, n, noalloc=True)[0]
    assert rc == F.FL_EINVAL
    assert _collect(srv, rid, n, noalloc=False)[0] == F.FL_OK
    srv.close()
