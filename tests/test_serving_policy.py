"""Admission order of the serving loop (host logic, no GPU): a stand-in server
with a fixed number of slots records the order in which requests are offered
and admitted; every admitted request finishes after a number of ticks equal to
its lattice length / 64."""
import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import serving
from paper_2212_10680_amd import workloads as wl


class StandInServer:
    def __init__(self, slots):
        self.slots = slots
        self.live = {}       # id -> (L, ticks left)
        self.admitted = []   # L in admission order
        self.finished = []
        self.next_id = 1

    def submit(self, rho0, shape, tol, check_every, max_steps):
        if len(self.live) >= self.slots:
            return None
        rid = self.next_id
        self.next_id += 1
        self.live[rid] = [shape[0], shape[0] // 64]
        self.admitted.append(shape[0])
        return rid

    def tick(self, max_steps, tick_ms):
        for rid, v in list(self.live.items()):
            v[1] -= 1
            if v[1] <= 0:
                self.finished.append(rid)

    def poll(self):
        out, self.finished = self.finished, []
        for rid in out:
            del self.live[rid]
        return out

    def result(self, rid, n):
        return np.zeros(n), 100, 0.0, F.FL_OK


@pytest.fixture(scope="module")
def reqs():
    return wl.serving_requests(n=24, seed=3)[0]


def test_largest_first_admits_longest_lattices_first(reqs):
    srv = StandInServer(slots=4)
    out = serving.serve(srv, reqs, np.zeros(len(reqs)), 1e-10, 1000, 50000, policy="largest_first")
    assert out["completed"] == len(reqs)
    assert srv.admitted == sorted((r["L"] for r in reqs), reverse=True)


def test_fifo_keeps_arrival_order(reqs):
    srv = StandInServer(slots=4)
    arrivals = np.linspace(0.0, 0.01, len(reqs))[::-1].copy()  # last request arrives first
    out = serving.serve(srv, reqs, arrivals, 1e-10, 1000, 50000, policy="fifo")
    assert out["completed"] == len(reqs)
    assert srv.admitted == [r["L"] for r in reqs[::-1]]


def test_largest_first_never_admits_before_arrival(reqs):
    """Only arrived requests are ranked: a long lattice arriving late does not
    overtake short ones that are already admitted."""
    srv = StandInServer(slots=64)
    arrivals = np.zeros(len(reqs))
    big = int(np.argmax([r["L"] for r in reqs]))
    arrivals[big] = 0.05
    serving.serve(srv, reqs, arrivals, 1e-10, 1000, 50000, policy="largest_first")
    assert srv.admitted[-1] == reqs[big]["L"]
    rest = [r["L"] for k, r in enumerate(reqs) if k != big]
    assert srv.admitted[:-1] == sorted(rest, reverse=True)
