"""The z-marching collide/stream kernel (k_collide_zmarch) against the plain
one (k_collide_stream) and the oracle.

Both kernels run the same per-node expressions (stencil_force +
collide_push) and differ only in where the stencil values come from (LDS
rings and registers vs global memory), so they must agree bitwise; a wrong
slot, halo offset or register shift changes bits.  Shapes cover several
tiles in x and y, z-ranges that do not divide nz, a single plane, FP64 and
FP32 populations, BGK and MRT, and the two benchmark lattices.
"""
import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import workloads as wl

from _util import direction_map, oracle_for, rel, smooth_3d_field

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def solver(w, precision, tune):
    s = F.Solver(F.Params.from_workload(w, precision=precision))
    s.set_tuning(tune)
    return s


CASES = [
    ("binary_slab_3d", (64, 8, 5), "fp64", "BGK", 2),      # ragged last z-range
    ("binary_slab_3d", (128, 8, 9), "fp32", "BGK", 4),
    ("ternary_droplets_3d", (64, 12, 16), "fp32", "MRT", 16),
    ("ternary_droplets_3d", (64, 4, 7), "fp64", "MRT", 3),
    ("binary_slab_3d", (192, 8, 6), "fp32", "MRT", 5),
    ("binary_slab_3d", (64, 4, 1), "fp64", "BGK", 16),     # one plane
]


@pytest.mark.parametrize("zorder", [0, 1])
@pytest.mark.parametrize("rev", [0, 1])
@pytest.mark.parametrize("wname,shape,precision,coll,zlen", CASES)
def test_zmarch_equals_plain_bitwise(wname, shape, precision, coll, zlen, rev, zorder):
    """rev = 1 marches each z-range downward (the default when the passes
    alternate direction), rev = 0 upward; zorder 0 takes the workgroups in
    XCD-contiguous chunks, 1 in XCD y-bands."""
    w = wl.WORKLOADS[wname].scaled(shape)
    w.collision = coll
    w.u0 = 0.0
    if w.geometry == "two_droplets":
        w.geometry = "slab"
    announce(f"zmarch vs plain {wname} {shape} {precision} {coll} zlen={zlen} rev={rev} zorder={zorder}")
    rho, u = smooth_3d_field(w, amp=0.005)
    a = solver(w, precision, f"zmarch=1,zlen={zlen},rev={rev},zorder={zorder}")
    b = solver(w, precision, f"zmarch=0,rev={rev}")
    a.set_state(rho, u)
    b.set_state(rho, u)
    assert list(a.step_timed(2)) == ["k_moments_eos", "k_collide_zmarch"]
    assert list(b.step_timed(2)) == ["k_moments_eos", "k_collide_stream"]
    a.step(18)
    b.step(18)
    ga, gb = a.populations(), b.populations()
    print(f"  max |diff| {np.max(np.abs(ga - gb)):.3e}", flush=True)
    assert np.array_equal(ga, gb)
    assert np.array_equal(a.fields()["u"], b.fields()["u"])


def test_zmarch_fp64_vs_oracle():
    w = wl.WORKLOADS["ternary_droplets_3d"].scaled((64, 8, 6))
    w.geometry = "slab"
    w.u0 = 0.0
    w.precision = "fp64"
    announce("zmarch FP64 vs oracle")
    rho, u = smooth_3d_field(w)
    o = oracle_for(w)
    o.init(rho.reshape(3, -1))
    s = solver(w, "fp64", "zmarch=1,zlen=4")
    s.set_state(rho)
    assert list(s.step_timed(1)) == ["k_moments_eos", "k_collide_zmarch"]
    o.run(1)
    s.step(9)
    o.run(9)
    e, _ = F.lattice_table(w.lattice)
    err = rel(s.populations(), o.g[:, direction_map(w.lattice, e), :])
    er = rel(s.fields()["rho_molar"], o.fields()["rho_molar"])
    print(f"  pops {err:.2e} rho {er:.2e}", flush=True)
    assert err < 1e-12 and er < 1e-12


@pytest.mark.parametrize("wname", ["binary_slab_3d", "ternary_droplets_3d"])
def test_bench_lattices_zmarch_equals_plain(wname):
    """The benchmark lattices at full size (D3Q19 128^3 binary BGK and 256^3
    ternary MRT, FP32 populations): the z-marching kernel bitwise equal to the
    plain one after a few steps."""
    w = wl.WORKLOADS[wname]
    announce(f"bench lattice {wname} {w.shape}")
    rho, u = wl.initial_field(w)
    steps = 6 if w.shape[0] <= 128 else 3
    a = solver(w, "fp32", "zmarch=1")
    a.set_state(rho, u)
    assert list(a.step_timed(1)) == ["k_moments_eos", "k_collide_zmarch"]
    a.step(steps - 1)
    fa = a.fields()["rho_molar"]
    a.close()
    del a
    b = solver(w, "fp32", "zmarch=0")
    b.set_state(rho, u)
    assert list(b.step_timed(1)) == ["k_moments_eos", "k_collide_stream"]
    b.step(steps - 1)
    assert np.array_equal(fa, b.fields()["rho_molar"])


@pytest.mark.parametrize("wname,shape,precision,coll", [
    ("binary_slab_3d", (64, 8, 5), "fp32", "BGK"),
    ("ternary_droplets_3d", (24, 12, 7), "fp64", "MRT"),
])
def test_sweep_order_bitwise(wname, shape, precision, coll):
    """The order in which the passes visit the nodes (forward or reversed,
    XCD-contiguous or plain block order, plane-major or y-major inside z-slabs,
    any block size) changes no bit."""
    w = wl.WORKLOADS[wname].scaled(shape)
    w.collision = coll
    w.u0 = 0.0
    if w.geometry == "two_droplets":
        w.geometry = "slab"
    announce(f"sweep order {wname} {shape} {precision} {coll}")
    rho, u = smooth_3d_field(w, amp=0.005)
    ref = None
    for tune in ("rev=0,remap=1", "rev=1,remap=1", "rev=1,remap=0", "rev=0,remap=0",
                 "order=1,rev=1", "order=1,rev=0,remap=0", "order=1,k1block=64,k2block=256"):
        s = solver(w, precision, tune)
        s.set_state(rho, u)
        s.step(15)
        g = s.populations()
        s.close()
        if ref is None:
            ref = g
        assert np.array_equal(g, ref), tune


def _sphere(w, shape, R):
    rL, rV, _ = w.phase_densities()
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
    ind = 0.5 * (1 - np.tanh((r - R) / 2.0))
    return np.stack([rV[i] + (rL[i] - rV[i]) * ind for i in range(len(rL))])


ISO_CASES = [
    # workload, shape, precision, collision, zlen
    ("ternary_droplets_3d", (64, 12, 16), "fp32", "MRT", 16),
    ("ternary_droplets_3d", (128, 8, 11), "fp32", "MRT", 4),   # ragged last z-range, two tiles in x
    ("ternary_droplets_3d", (64, 8, 7), "fp64", "MRT", 3),
    ("ternary_droplets_3d", (64, 52, 6), "fp32", "MRT", 4),    # 13 tile rows: unequal XCD y-bands
    ("ternary_droplets_3d", (256, 12, 9), "fp32", "MRT", 4),   # four tiles in x, ragged z-range
    ("ternary_droplets_3d", (64, 8, 2), "fp32", "BGK", 16),    # two planes: z -+ 1 both the other one
    ("binary_slab_3d", (64, 8, 9), "fp32", "BGK", 2),
    ("binary_slab_3d", (64, 4, 1), "fp64", "BGK", 16),         # one plane: the three-pass form runs
    ("binary_slab_3d", (64, 4, 2), "fp32", "MRT", 1),          # two planes, one per workgroup
]


def iso_zmarch_name(ncomp, csplit):
    """The z-marching isotropic collide kernel a step runs: with three
    components each component gets its own 256 threads unless csplit=0."""
    return "k_collide_zmarch_iso_cs" if ncomp == 3 and csplit else "k_collide_zmarch_iso"


# csplit selects between the two forms only with three components; the others
# run the one-thread-per-node form with either value, so they take csplit=1 alone
ISO_RUNS = [case + (csplit, zorder) for case in ISO_CASES for csplit in (1, 0) for zorder in (0, 1)
            if csplit == 1 or wl.WORKLOADS[case[0]].ncomp == 3]


@pytest.mark.parametrize("wname,shape,precision,coll,zlen,csplit,zorder", ISO_RUNS)
def test_zmarch_isotropic_equals_plain_bitwise(wname, shape, precision, coll, zlen, csplit, zorder):
    """The z-marching kernel with the isotropic stencils (which forms
    -lap(phi) and mu_i in LDS as planes pass) against the one-thread-per-node
    kernel after the Laplacian pass: the same per-node expressions, so the
    same bits, on a droplet that varies along every axis.  With three
    components, both forms of the z-marching kernel: one thread per node
    (csplit=0) and one 256-thread group per component exchanging densities,
    momenta and forces through LDS (csplit=1); each in both block orders
    (zorder 0: XCD-contiguous chunks, 1: XCD y-bands)."""
    w = wl.WORKLOADS[wname].scaled(shape)
    w.collision = coll
    announce(f"iso zmarch vs plain {wname} {shape} {precision} {coll} zlen={zlen} csplit={csplit} "
             f"zorder={zorder}")
    rho = _sphere(w, shape, 0.3 * min(shape[:2]) if shape[2] > 2 else 1.5)
    p = F.Params.from_workload(w, precision=precision, stencil="isotropic")
    a, b = F.Solver(p), F.Solver(p)
    a.set_tuning(f"zmarch=1,zlen={zlen},csplit={csplit},zorder={zorder}")
    b.set_tuning("zmarch=0")
    a.set_state(rho)
    b.set_state(rho)
    plain = {"k_moments_eos", "k_collide_stream", "k_interface_lap"}
    if shape[2] >= 2:
        assert list(a.step_timed(1)) == ["k_moments_eos", iso_zmarch_name(w.ncomp, csplit)]
    else:  # one plane: the isotropic z-march needs two, the three-pass form runs
        assert set(a.step_timed(1)) == plain
    assert set(b.step_timed(1)) == plain
    a.step(14)
    b.step(14)
    ga, gb = a.populations(), b.populations()
    print(f"  max |diff| {np.max(np.abs(ga - gb)):.3e}", flush=True)
    assert np.array_equal(ga, gb)
    assert np.array_equal(a.fields()["u"], b.fields()["u"])
    a.close()
    b.close()


@pytest.mark.parametrize("csplit", [0, 1])
def test_zmarch_isotropic_fp64_vs_oracle(csplit):
    """FP64 z-marching isotropic kernel (both forms) against the oracle's
    isotropic form on a ternary sphere (MRT), element by element (1e-12)."""
    shape = (64, 12, 10)
    w = wl.WORKLOADS["ternary_droplets_3d"].scaled(shape)
    announce(f"iso zmarch FP64 vs oracle {shape} csplit={csplit}")
    rho = _sphere(w, shape, 4.0).reshape(3, -1)
    o = oracle_for(w, stencil="isotropic")
    o.init(rho)
    s = F.Solver(F.Params.from_workload(w, precision="fp64", stencil="isotropic"))
    # three components in FP64 default to the one-thread-per-node form; both
    # are asked for
    s.set_tuning(f"zmarch=1,csplit={csplit}")
    s.set_state(rho)
    assert list(s.step_timed(1)) == ["k_moments_eos", iso_zmarch_name(3, csplit)]
    o.run(1)
    s.step(29)
    o.run(29)
    e, _ = F.lattice_table(w.lattice)
    err = rel(s.populations(), o.g[:, direction_map(w.lattice, e), :])
    er = rel(s.fields()["rho_molar"], o.fields()["rho_molar"])
    print(f"  pops {err:.2e} rho {er:.2e}", flush=True)
    assert err < 1e-12 and er < 1e-12


def test_bench_lattice_isotropic_zmarch_equals_plain():
    """The 256^3 ternary two-droplet lattice of the benchmark (FP32, MRT,
    isotropic stencils): both z-marching forms and the one-thread-per-node
    kernel bitwise equal after three steps."""
    w = wl.WORKLOADS["ternary_droplets_3d"]
    announce(f"bench lattice isotropic {w.shape}")
    rho, u = wl.initial_field(w)
    out = []
    for tune in ("zmarch=1", "zmarch=1,csplit=0", "zmarch=0", "zmarch=1,zorder=1,zlen=8",
                 "zmarch=1,csplit=0,zorder=1,zlen=4", "zmarch=1,zorder=0", "zmarch=1,remap=1,k1block=128"):
        s = F.Solver(F.Params.from_workload(w, precision="fp32", stencil="isotropic"))
        s.set_tuning(tune)
        s.set_state(rho, u)
        s.step(3)
        out.append(s.fields()["rho_molar"])
        s.close()
        del s
    for o in out[1:]:
        assert np.array_equal(out[0], o)
