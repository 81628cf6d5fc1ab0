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

    def result(self, rid, n, full=False):
        if full:
            return {"rho_molar": np.zeros(n), "u": np.zeros(n), "p": np.zeros(n), "steps": 100,
                    "residual": 0.0, "status": F.FL_OK, "latency_s": 0.0}
        return np.zeros(n), 100, 0.0, F.FL_OK


@pytest.fixture(scope="module")
def reqs():
    return wl.serving_requests(n=24, seed=3)[0]


def test_largest_first_admits_longest_lattices_first(reqs):
    srv = StandInServer(slots=4)
    out = serving.serve(srv, reqs, np.zeros(len(reqs)), 1e-10, 1000, 50000, policy="largest_first")
    assert out["completed"] == out["converged"] == len(reqs)
    assert out["converged_solves_per_s"] > 0 and out["p99_time_to_equilibrium_s"] >= 0
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


def test_metrics_count_converged_requests_only(reqs):
    """Requests stopped at max_steps or by a numeric failure are reported but
    enter neither the throughput nor the time-to-equilibrium percentiles."""

    class Mixed(StandInServer):
        def result(self, rid, n, full=False):
            st = (F.FL_OK, F.FL_ENOTCONV, F.FL_ENUMERIC)[rid % 3]
            return {"rho_molar": np.zeros(n), "u": np.zeros(n), "p": np.zeros(n), "steps": 100,
                    "residual": 0.0, "status": st, "latency_s": 0.0}

    srv = Mixed(slots=64)
    out = serving.serve(srv, reqs, np.zeros(len(reqs)), 1e-10, 1000, 50000)
    conv = [r for r in out["records"] if r["status"] == F.FL_OK]
    assert out["completed"] == len(reqs)
    assert out["converged"] == len(conv) == len(reqs) // 3
    assert out["max_steps_reached"] == out["numeric_failures"] == len(reqs) // 3
    span = max(r["done"] for r in out["records"]) - min(r["arrival"] for r in out["records"])
    assert abs(out["converged_solves_per_s"] - len(conv) / span) < 1e-9 * out["converged_solves_per_s"]
    assert out["p99_time_to_equilibrium_s"] <= max(r["latency"] for r in conv) + 1e-12
