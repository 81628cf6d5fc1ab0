"""The fused one-launch step (k_fused_step) against the two-kernel step and the oracle.

Both paths run the same per-node arithmetic, so any stale read of the
densities or ln f inside the fused launch (a dependency or cache-coherence
mistake) changes bits: the comparison is bitwise.  Shapes cover ragged
256-node tiles, planes that do not split evenly over the 8 XCDs, FP64 and
FP32 populations, BGK and MRT, and the full benchmark sizes.
"""
import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import workloads as wl

from _util import direction_map, oracle_for, rel, smooth_3d_field

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def solver(w, precision, fused):
    s = F.Solver(F.Params.from_workload(w, precision=precision))
    s.set_tuning("fused=1" if fused else "fused=0")
    return s


def field(w):
    if w.D == 3:
        return smooth_3d_field(w, amp=0.005)
    rho, u = wl.initial_field(w)
    nx, ny = w.shape
    y = np.arange(ny)[:, None]
    return np.ascontiguousarray(rho * (1 + 0.005 * np.sin(2 * np.pi * y / ny))[None, None]), u


def pair(w, precision):
    rho, u = field(w)
    a, b = solver(w, precision, True), solver(w, precision, False)
    a.set_state(rho, u)
    b.set_state(rho, u)
    return a, b


CASES = [
    ("binary_slab_3d", (32, 64, 16), "fp32", "BGK"),
    ("binary_slab_3d", (48, 72, 9), "fp64", "BGK"),       # 9 rows per XCD: ragged tile
    ("ternary_droplets_3d", (16, 67, 12), "fp32", "MRT"),  # 67 rows: uneven split over XCDs
    ("ternary_droplets_3d", (32, 64, 20), "fp64", "MRT"),
    ("binary_slab_3d", (16, 96, 5), "fp64", "MRT"),        # thin sweep axis (z wraps fast)
]


@pytest.mark.parametrize("wname,shape,precision,coll", CASES)
def test_fused_equals_two_kernel_bitwise(wname, shape, precision, coll):
    w = wl.WORKLOADS[wname].scaled(shape)
    w.collision = coll
    w.u0 = 0.0
    if w.geometry == "two_droplets":
        w.geometry = "slab"
    announce(f"fused vs two-kernel {wname} {shape} {precision} {coll}")
    a, b = pair(w, precision)
    ka = a.step_timed(3)
    kb = b.step_timed(3)
    assert list(ka) == ["k_fused_step"] and list(kb) == ["k_moments_eos", "k_collide_stream"]
    a.step(17)
    b.step(17)
    ga, gb = a.populations(), b.populations()
    print(f"  max |diff| {np.max(np.abs(ga - gb)):.3e}", flush=True)
    assert np.array_equal(ga, gb)
    assert np.array_equal(a.fields()["u"], b.fields()["u"])


def test_fused_fp64_vs_oracle():
    w = wl.WORKLOADS["ternary_droplets_3d"].scaled((16, 64, 12))
    w.geometry = "slab"
    w.u0 = 0.0
    w.precision = "fp64"
    announce("fused FP64 vs oracle")
    rho, u = smooth_3d_field(w)
    o = oracle_for(w)
    o.init(rho.reshape(3, -1))
    s = solver(w, "fp64", True)
    s.set_state(rho)
    assert list(s.step_timed(1)) == ["k_fused_step"]
    o.run(1)
    s.step(9)
    o.run(9)
    e, _ = F.lattice_table(w.lattice)
    g = s.populations()
    err = rel(g, o.g[:, direction_map(w.lattice, e), :])
    er = rel(s.fields()["rho_molar"], o.fields()["rho_molar"])
    print(f"  pops {err:.2e} rho {er:.2e}", flush=True)
    assert err < 1e-12 and er < 1e-12


def test_bench_size_fused_vs_two_kernel_and_oracle_columns():
    """Full benchmark configuration (D3Q19 128^3 binary slab, FP32 populations):
    fused == two-kernel bitwise, every (y, z) column identical (the slab stays
    uniform along y and z), and the columns within 1e-4 of the FP64 oracle run
    on a 128 x 2 x 2 lattice, which is the same problem."""
    w = wl.WORKLOADS["binary_slab_3d"]
    announce("bench size 128^3")
    rho, u = wl.initial_field(w)
    a, b = solver(w, "fp32", True), solver(w, "fp32", False)
    a.set_state(rho)
    b.set_state(rho)
    a.step(50)
    b.step(50)
    fa = a.fields()["rho_molar"]
    assert np.array_equal(fa, b.fields()["rho_molar"])
    cols = fa.reshape(2, 128, 128, 128)
    assert np.array_equal(cols, np.broadcast_to(cols[:, :1, :1, :], cols.shape))
    ws = w.scaled((128, 2, 2))
    o = oracle_for(ws)
    r2, _ = wl.initial_field(ws)
    o.init(r2.reshape(2, -1))
    o.run(50)
    ref = o.fields()["rho_molar"].reshape(2, 2, 2, 128)[:, 0, 0, :]
    err = rel(cols[:, 0, 0, :], ref)
    print(f"  column vs oracle {err:.2e}", flush=True)
    assert err < 1e-4


def test_largest_config_fused_vs_two_kernel():
    """D3Q19 256^3 ternary MRT, FP32 populations (7.6 GB of populations per
    solver): a few steps bitwise equal between the two paths."""
    w = wl.WORKLOADS["ternary_droplets_3d"]
    announce("256^3 ternary")
    rho, u = wl.initial_field(w)
    a = solver(w, "fp32", True)
    a.set_state(rho, u)
    a.step(4)
    ga = a.fields()["rho_molar"]
    a.close()
    del a
    b = solver(w, "fp32", False)
    b.set_state(rho, u)
    b.step(4)
    assert np.array_equal(ga, b.fields()["rho_molar"])
