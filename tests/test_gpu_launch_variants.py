"""Launch choices that must not change a result bit (fl_set_tuning).

The XCD-band visiting order of the plain collide pass and of the interface
Laplacian pass only changes which workgroup computes which node: every node's
arithmetic is the same, so the populations must agree bitwise with the plain
order.  Shapes have ny not divisible by the band count, so some bands are a
row narrower, and (with 16 or 32 bands) fewer rows than bands per XCD sweep.
"""
import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import workloads as wl

from _util import smooth_3d_field

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def _sphere_pair(w, shape, R):
    rL, rV, _ = w.phase_densities()
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
    ind = 0.5 * (1 - np.tanh((r - R) / 2.0))
    return np.stack([rV[i] + (rL[i] - rV[i]) * ind for i in range(len(rL))]).reshape(len(rL), -1)


CASES = [
    # workload, shape, precision, stencil, tuning
    ("ternary_droplets_3d", (40, 35, 12), "fp32", "isotropic", "bands=8,lapbands=8"),
    ("ternary_droplets_3d", (40, 35, 12), "fp64", "isotropic", "bands=16,lapbands=32"),
    ("binary_slab_3d", (26, 21, 10), "fp32", "isotropic", "bands=32"),
    ("binary_slab_3d", (26, 21, 10), "fp64", "axis", "zmarch=0,bands=8"),
    ("ternary_droplets_3d", (30, 17, 7), "fp32", "axis", "bands=16,rev=1"),
]


@pytest.mark.parametrize("wname,shape,precision,stencil,tune", CASES)
def test_band_order_bitwise(wname, shape, precision, stencil, tune):
    w = wl.WORKLOADS[wname].scaled(shape)
    announce(f"band order {wname} {shape} {precision} {stencil} {tune}")
    if stencil == "isotropic":
        rho, u = _sphere_pair(w, shape, 6.0), None
    else:
        w.geometry = "slab"
        w.u0 = 0.0
        rho, u = smooth_3d_field(w)
    p = F.Params.from_workload(w, precision=precision, stencil=stencil)
    a, b = F.Solver(p), F.Solver(p)
    b.set_tuning(tune)
    a.set_state(rho, u)
    b.set_state(rho, u)
    names = b.step_timed(1)
    a.step(1)
    assert "k_collide_stream" in names, names
    a.step(19)
    b.step(19)
    ga, gb = a.populations(), b.populations()
    print(f"  max |diff| {np.max(np.abs(ga - gb)):.1e}", flush=True)
    assert np.array_equal(ga, gb)
    a.close()
    b.close()


PAIR_CASES = [
    # workload, shape, precision, stencil: two nodes per thread in the moments
    # pass where it applies (N_c >= 3, FP32, N even), else the one-node form
    ("ternary_droplets_3d", (64, 8, 6), "fp32", "isotropic"),   # z-marching collide pass
    ("ternary_droplets_3d", (40, 35, 12), "fp32", "axis"),      # plain collide pass
    ("ternary_droplets_3d", (33, 17, 7), "fp32", "isotropic"),  # N odd: one node per thread
    ("ternary_droplet_2d", (64, 30), "fp32", "axis"),           # D2Q9
    ("ternary_droplets_3d", (64, 8, 6), "fp64", "isotropic"),   # FP64: one node per thread
]


@pytest.mark.parametrize("wname,shape,precision,stencil", PAIR_CASES)
def test_moments_pair_bitwise(wname, shape, precision, stencil):
    """The moments pass with two consecutive nodes per thread (mpair=1, the
    default) runs each node's arithmetic unchanged, so every field and every
    population after 20 steps is the same bit for bit as with one node per
    thread (mpair=0)."""
    w = wl.WORKLOADS[wname].scaled(shape)
    announce(f"moments pair {wname} {shape} {precision} {stencil}")
    if w.lattice == "D2Q9":  # a disc droplet
        rL, rV, _ = w.phase_densities()
        nx, ny = shape
        y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2)
        ind = 0.5 * (1 - np.tanh((r - 8.0) / 2.0))
        rho = np.stack([rV[i] + (rL[i] - rV[i]) * ind for i in range(len(rL))]).reshape(len(rL), -1)
        u = None
    else:
        rho, u = _sphere_pair(w, shape, min(shape[0], shape[1]) / 3.0), None
    p = F.Params.from_workload(w, precision=precision, stencil=stencil)
    a, b = F.Solver(p), F.Solver(p)
    # the two-node form runs with 256-thread blocks in plain order, the
    # defaults of the isotropic three-component lattices; set them everywhere
    a.set_tuning("k1block=256,remap=0")
    b.set_tuning("k1block=256,remap=0,mpair=0")
    a.set_state(rho, u)
    b.set_state(rho, u)
    a.step(20)
    b.step(20)
    ga, gb = a.populations(), b.populations()
    print(f"  max |diff| {np.max(np.abs(ga - gb)):.1e}", flush=True)
    assert np.array_equal(ga, gb)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    a.close()
    b.close()


def test_tuning_rejects_unknown_keys_and_values():
    w = wl.WORKLOADS["binary_slab_3d"].scaled((16, 8, 4))
    s = F.Solver(F.Params.from_workload(w, precision="fp32"))
    for bad in ("bands=12", "k2block=100", "nosuchkey=1", "zmarch=2", "csplit=3", "zorder=2", "mpair=2", "bands", "bands=8x"):
        with pytest.raises(F.FLError) as ei:
            s.set_tuning(bad)
        assert ei.value.status == F.FL_EINVAL
    s.set_tuning("bands=8, k2block=64, csplit=0, zorder=1, mpair=0".replace(" ", ""))
    s.set_tuning(None)
    s.close()
