"""GPU (HIP, gfx950) parity with the FP64 oracle, through the C ABI.

FP64 path: populations and fields element by element after 1, 10 and 1000
steps, bar 1e-12 relative (oracle transients are "parity unpinned" beyond the
oracle itself, so the bar is rounding-level agreement).  FP32-population form:
densities within 1e-4 relative of the FP64 oracle (the stated tolerance for the
precision form).  Sizes span several 256-node blocks and a ragged tail.
"""
import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import workloads as wl

from _util import (bulk_values, direction_map, flash_errors_percent, mixture_of, oracle_for, rel,
                   smooth_3d_field)

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-12
FP32_BAR = 1e-4


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def make_pair(w, precision="fp64", rho=None, u=None, force_level=0, eos="PR", mrt_rates=None,
              stencil="axis"):
    if rho is None:
        rho, u = wl.initial_field(w)
    nc, D = w.ncomp, w.D
    rho = rho.reshape(nc, -1)
    u = None if u is None else u.reshape(D, -1)
    S = None
    if mrt_rates is not None:
        from oracle import lattice as olat
        _, groups = olat.mrt_basis(w.lattice)
        table = {"rho": 1.0 / w.tau, "j": mrt_rates[0], "nu": mrt_rates[1], "e": mrt_rates[2],
                 "ghost": mrt_rates[3]}
        S = np.array([table[g] for g in groups])
    o = oracle_for(w, eos=eos, force_level=force_level, mrt_S=S, stencil=stencil)
    o.init(rho, u)
    p = F.Params.from_workload(w, precision=precision, force_time_level=force_level, eos=eos,
                               mrt_rates=mrt_rates, stencil=stencil)
    s = F.Solver(p)
    s.set_state(rho, u)
    return o, s


def compare(o, s, w, bar, what=""):
    e, _ = F.lattice_table(w.lattice)
    perm = direction_map(w.lattice, e)
    g_gpu = s.populations()
    g_orc = o.g[:, perm, :]
    eg = rel(g_gpu, g_orc)
    fo = o.fields()
    fs = s.fields()
    er = rel(fs["rho_molar"], fo["rho_molar"])
    eu = float(np.max(np.abs(fs["u"] - fo["u"])) / max(np.max(np.abs(fo["u"])), 1e-12))
    ep = rel(fs["p"], fo["p"])
    el = rel(fs["lnf"], fo["lnf"])
    print(f"  {what} steps={o.steps}: pops {eg:.2e} rho {er:.2e} u {eu:.2e} p {ep:.2e} lnf {el:.2e}",
          flush=True)
    assert eg < bar and er < bar and ep < bar and el < bar, (eg, er, ep, el)
    assert eu < max(bar * 1e3, 1e-9) if bar < 1e-6 else eu < 1e-2
    return eg


CASES_FP64 = [
    # name, workload, shape, steps schedule
    ("binary D2Q9 BGK noisy 61x7", "binary_slab_2d", (61, 7), (1, 9, 990)),
    ("binary D2Q9 BGK 64x8 (cfg0 shape)", "binary_slab_2d", (64, 8), (1, 9, 990)),
    ("ternary D2Q9 MRT droplet 48x40", "ternary_droplet_2d", (48, 40), (1, 9, 190)),
]


@pytest.mark.parametrize("name,wname,shape,sched", CASES_FP64)
def test_fp64_parity_2d(name, wname, shape, sched):
    w = wl.WORKLOADS[wname].scaled(shape)
    announce(name)
    o, s = make_pair(w)
    for k in sched:
        o.run(k)
        s.step(k)
        compare(o, s, w, FP64_BAR, name)


@pytest.mark.parametrize("coll", ["BGK", "MRT"])
@pytest.mark.parametrize("wname,shape", [("binary_slab_3d", (21, 10, 6)),
                                         ("ternary_droplets_3d", (20, 12, 9))])
def test_fp64_parity_3d(coll, wname, shape):
    w = wl.WORKLOADS[wname].scaled(shape)
    w.collision = coll
    if wname == "ternary_droplets_3d":
        w.geometry = "slab"          # smooth 3-D field (see smooth_3d_field)
        w.u0 = 0.0
    rho, u = smooth_3d_field(w)
    announce(f"{wname} D3Q19 {coll} {shape}")
    o, s = make_pair(w, rho=rho, u=u)
    # short runs: D3Q19 fields grow high-wavenumber modes, which amplify any
    # rounding difference by about x200 every further 10 steps
    for k in (1, 9):
        o.run(k)
        s.step(k)
        compare(o, s, w, FP64_BAR, f"3d {coll}")


def _sphere(w, shape, R):
    """Droplet of radius R (tanh profile of width 2) centred in the box."""
    rL, rV, _ = w.phase_densities()
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
    ind = 0.5 * (1 - np.tanh((r - R) / 2.0))
    return np.stack([rV[i] + (rL[i] - rV[i]) * ind for i in range(len(rL))]).reshape(len(rL), -1)


@pytest.mark.parametrize("coll", ["BGK", "MRT"])
def test_isotropic_stencils_sphere_vs_oracle(coll):
    """The isotropic lattice stencils (the option that keeps 3-D droplets in
    the EOS domain) on a D3Q19 sphere of the benchmark's binary mixture:
    FP64 element by element against the oracle's isotropic form, on a box
    that is not a multiple of the z-marching tile in x (so the plain kernel
    and the Laplacian pass run)."""
    shape = (26, 24, 20)
    w = wl.WORKLOADS["binary_slab_3d"].scaled(shape)
    w.collision = coll
    rho = _sphere(w, shape, 6.0)
    announce(f"isotropic stencils D3Q19 {coll} sphere {shape}")
    o, s = make_pair(w, rho=rho, stencil="isotropic")
    for k in (1, 9, 40):
        o.run(k)
        s.step(k)
        compare(o, s, w, FP64_BAR, f"iso 3d {coll}")
    # a box whose x extent is a multiple of 64 and y of 4 takes the z-marching
    # form, which computes -lap(phi) itself (no Laplacian pass)
    w2 = wl.WORKLOADS["binary_slab_3d"].scaled((64, 8, 8))
    p = F.Params.from_workload(w2, precision="fp32", stencil="isotropic")
    s2 = F.Solver(p)
    s2.set_state(*wl.initial_field(w2))
    names = s2.step_timed(2)
    assert list(names) == ["k_moments_eos", "k_collide_zmarch_iso"], names


def test_isotropic_stencils_2d_and_fp32():
    """D2Q9 ternary MRT droplet with the isotropic stencils (FP64, 1e-12), and
    the FP32-population form on the 3-D sphere (1e-4 of the FP64 oracle)."""
    w = wl.WORKLOADS["ternary_droplet_2d"].scaled((48, 40))
    announce("isotropic stencils D2Q9 ternary MRT droplet 48x40")
    o, s = make_pair(w, stencil="isotropic")
    for k in (1, 9, 90):
        o.run(k)
        s.step(k)
        compare(o, s, w, FP64_BAR, "iso 2d")
    shape = (26, 24, 20)
    w3 = wl.WORKLOADS["binary_slab_3d"].scaled(shape)
    announce(f"isotropic stencils D3Q19 FP32 sphere {shape}")
    o, s = make_pair(w3, precision="fp32", rho=_sphere(w3, shape, 6.0), stencil="isotropic")
    o.run(50)
    s.step(50)
    fo, fs = o.fields(), s.fields()
    assert rel(fs["rho_molar"], fo["rho_molar"]) < FP32_BAR


def test_isotropic_stencils_coalescence_256():
    """The 256^3 ternary two-droplet lattice (radius 30, centres 70 apart,
    approaching at +-0.02, MRT tau 0.8, FP32 populations) with the isotropic
    stencils: with the axis stencils it leaves the EOS domain within 50 steps;
    here it stays in the domain, the neck between the droplets fills with
    liquid (the droplets coalesce) and each component's mass is conserved."""
    w = wl.WORKLOADS["ternary_droplets_3d"]
    rL, rV, _ = w.phase_densities()
    L, V = float(np.sum(rL)), float(np.sum(rV))
    n = w.shape[0]
    c = n // 2
    rho, u = wl.initial_field(w)
    mid0 = float(rho[:, c, c, c].sum())
    assert mid0 < V + 0.5 * (L - V), mid0     # vapour between the droplets at the start
    announce("isotropic stencils: 256^3 ternary coalescence, 1000 steps")
    s = F.Solver(F.Params.from_workload(w, stencil="isotropic"))
    s.set_state(rho, u)
    m0 = s.mass()
    s.step(1000)
    f = s.fields()
    r = f["rho_molar"].sum(0).reshape(n, n, n)
    dm = np.abs(s.mass() - m0) / m0
    um = float(np.abs(f["u"]).max())
    print(f"  mid {mid0:.3f} -> {r[c, c, c]:.3f} (L {L:.3f} V {V:.3f}) |u|max {um:.2e} mass drift {dm}",
          flush=True)
    assert r[c, c, c] > V + 0.9 * (L - V)       # liquid neck
    assert np.all(dm < 1e-8)
    assert um < 0.05
    assert 0.9 * V < r.min() and r.max() < 1.1 * L


@pytest.mark.parametrize("wname,precision,stencil", [
    ("ternary_droplets_3d", "fp64", "axis"),
    ("ternary_droplets_3d", "fp64", "isotropic"),
    ("ternary_droplets_3d", "fp32", "isotropic"),
    ("binary_slab_3d", "fp32", "axis"),
])
def test_full_size_one_step_sampled_vs_oracle(wname, precision, stencil):
    """The 3-D benchmark lattices at full size (256^3 ternary two droplets, MRT
    tau 0.8; 128^3 binary slab, BGK), one step, in the launch configuration
    the benchmark times (FP32 populations) and in FP64: a node's fields after
    one step depend on the state within 3 nodes of it (moments and EOS local,
    forces from radius 2, the interface Laplacian one node further).  So the
    oracle runs one step on 17^3 periodic windows of the same initial state
    around sampled nodes (the neck between the droplets, interfaces, the
    wrapped corner), and its central 9^3 nodes must match the GPU's
    full-lattice result element by element (FP64 1e-12, FP32 1e-4)."""
    w = wl.WORKLOADS[wname]
    n = w.shape[0]
    nc = w.ncomp
    bar, ubar = (FP64_BAR, 1e-9) if precision == "fp64" else (FP32_BAR, 1e-2)
    rho, u = wl.initial_field(w)
    if u is None:
        u = np.zeros((3,) + rho.shape[1:])
    announce(f"full size one step, {wname} {w.shape} {precision}, {stencil} stencils")
    s = F.Solver(F.Params.from_workload(w, precision=precision, stencil=stencil))
    s.set_state(rho, u)
    s.step(1)
    fs = s.fields()
    s.close()
    del s
    gr = fs["rho_molar"].reshape(nc, n, n, n)
    gu = fs["u"].reshape(3, n, n, n)
    gl = fs["lnf"].reshape(nc, n, n, n)
    h, k = 8, 4
    q = n // 2
    # (z, y, x): centre, interfaces of the droplets / the slab, the wrapped corner
    samples = [(q, q, q), (q, q, q - 65 * n // 256), (q, q - 28 * n // 256, q - 35 * n // 256), (0, 0, 0)]
    if wname == "binary_slab_3d":
        samples = [(q, q, n // 4), (q, 5, 3 * n // 4), (n - 3, q, q), (0, 0, 0)]
    for c in samples:
        idx = [np.arange(c[d] - h, c[d] + h + 1) % n for d in range(3)]
        win = np.ix_(idx[0], idx[1], idx[2])
        o = oracle_for(w.scaled((2 * h + 1,) * 3), stencil=stencil)
        o.init(np.stack([r[win] for r in rho]).reshape(nc, -1), np.stack([v[win] for v in u]).reshape(3, -1))
        o.run(1)
        fo = o.fields()
        m = 2 * h + 1
        sl = (slice(h - k, h + k + 1),) * 3
        inner = np.ix_(*[idx[d][h - k:h + k + 1] for d in range(3)])
        er = rel(gr[(slice(None),) + inner], fo["rho_molar"].reshape(nc, m, m, m)[(slice(None),) + sl])
        el = rel(gl[(slice(None),) + inner], fo["lnf"].reshape(nc, m, m, m)[(slice(None),) + sl])
        ou = fo["u"].reshape(3, m, m, m)[(slice(None),) + sl]
        # far from the droplets u is zero up to rounding, and a momentum sum of
        # O(1) populations carries ~1e-15 of absolute rounding: u is scaled by
        # at least 1e-3 (the approach speed is 0.02)
        eu = float(np.max(np.abs(gu[(slice(None),) + inner] - ou)) / max(np.max(np.abs(ou)), 1e-3))
        print(f"  sample {c}: rho {er:.2e} lnf {el:.2e} u {eu:.2e}", flush=True)
        assert er < bar and el < bar and eu < ubar, (c, er, el, eu)


def test_server_rejects_isotropic_stencils():
    w = wl.WORKLOADS["binary_slab_3d"]
    p = F.Params.from_workload(w, precision="fp64", stencil="isotropic")
    with pytest.raises(F.FLError):
        F.Server(p, 1 << 20)


def smooth_vapor_field(w, rho_V, amp=0.05):
    """Single-phase vapor-like field with smooth, component-shifted modulations:
    exercises every term of the step without the interface instabilities."""
    nx, ny = w.shape[0], w.shape[1]
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    for i, r in enumerate(rho_V):
        out.append(r * (1 + amp * np.sin(2 * np.pi * (x / nx + 0.1 * i))
                        + 0.6 * amp * np.cos(2 * np.pi * (y / ny + 0.2 * i))))
    return np.ascontiguousarray(np.stack(out)[:, None])


@pytest.mark.parametrize("variant", ["force_level_1", "SRK", "VDW", "mrt_all_rates"])
def test_fp64_parity_variants(variant):
    w = wl.WORKLOADS["binary_slab_2d"].scaled((40, 6))
    kw = {}
    if variant == "force_level_1":
        kw["force_level"] = 1
    elif variant in ("SRK", "VDW"):
        kw["eos"] = variant
    else:
        w.collision = "MRT"
        kw["mrt_rates"] = [1.1, 0.9, 1.2, 1.3]
    _, rV, _ = w.phase_densities()
    rho = smooth_vapor_field(w, rV)
    announce(f"variant {variant}")
    o, s = make_pair(w, rho=rho, **kw)
    for k in (1, 99):
        o.run(k)
        s.step(k)
        compare(o, s, w, FP64_BAR, variant)


@pytest.mark.parametrize("nc", [1, 4])
def test_fp64_parity_component_counts(nc):
    """One component (pure fluid) and four components (the ABI maximum)."""
    base = wl.WORKLOADS["ternary_droplet_2d"].scaled((33, 9))
    comps, kij, T = base.thermo()
    if nc == 1:
        comps = [comps[2]]
        kij = np.zeros((1, 1))
    else:
        extra = dict(comps[1])
        extra["Tc"] *= 1.1
        extra["Pc"] *= 1.05
        comps = comps + [extra]
        kij = np.pad(kij, ((0, 1), (0, 1)), constant_values=0.01)
        np.fill_diagonal(kij, 0.0)
    from oracle import lbm, thermo as th
    mix = th.Mixture([c["Tc"] for c in comps], [c["Pc"] for c in comps], [c["omega"] for c in comps],
                     T, kij=kij, M=[c["M"] for c in comps], kappa=[c["kappa"] for c in comps])
    nx, ny = base.shape
    rho = smooth_vapor_field(base, [0.3 + 0.1 * k for k in range(nc)]).reshape(nc, -1)
    o = lbm.OracleLBM(mix, "D2Q9", (nx, ny), tau=1.0)
    o.init(rho)
    p = F.Params(comps, T, (nx, ny), kij=kij, tau=1.0)
    announce(f"nc={nc}")
    s = F.Solver(p)
    s.set_state(rho)
    for k in (1, 99):
        o.run(k)
        s.step(k)
        compare(o, s, base, FP64_BAR, f"nc={nc}")


@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (7, 1), (2, 3)])
def test_degenerate_shapes(shape):
    """Lattices thinner than the stencil (periodic images coincide)."""
    w = wl.WORKLOADS["binary_slab_2d"].scaled(shape)
    w.noise = 0.003
    announce(f"degenerate {shape}")
    rL, rV, _ = w.phase_densities()
    rho, _ = wl.initial_field(w, rho_LV=(0.5 * (rL + rV), 0.5 * (rL + rV)))
    o, s = make_pair(w, rho=rho)
    o.run(20)
    s.step(20)
    compare(o, s, w, FP64_BAR, f"degenerate {shape}")


def test_fp32_form_vs_oracle():
    """FP32 populations + FP64 EOS: densities within 1e-4 of the FP64 oracle."""
    w = wl.WORKLOADS["binary_slab_2d"].scaled((64, 8))
    announce("fp32 form 64x8")
    o, s = make_pair(w, precision="fp32")
    for k in (1, 999):
        o.run(k)
        s.step(k)
        fo, fs = o.fields(), s.fields()
        er = rel(fs["rho_molar"], fo["rho_molar"])
        ep = rel(fs["p"], fo["p"])
        print(f"  fp32 steps={o.steps}: rho {er:.2e} p {ep:.2e}", flush=True)
        assert er < FP32_BAR and ep < FP32_BAR


def test_fp32_form_3d_mrt():
    w = wl.WORKLOADS["ternary_droplets_3d"].scaled((20, 12, 9))
    w.geometry = "slab"
    w.u0 = 0.0
    rho, u = smooth_3d_field(w)
    announce("fp32 form D3Q19 MRT ternary")
    o, s = make_pair(w, precision="fp32", rho=rho, u=u)
    o.run(20)
    s.step(20)
    er = rel(s.fields()["rho_molar"], o.fields()["rho_molar"])
    print(f"  rho {er:.2e}", flush=True)
    assert er < FP32_BAR


# --------------------------------------------------------------- invariants
def test_mass_conservation_and_determinism():
    w = wl.WORKLOADS["binary_slab_2d"].scaled((64, 8))
    announce("mass + determinism")
    rho, u = wl.initial_field(w)
    p = F.Params.from_workload(w)
    a, b = F.Solver(p), F.Solver(p)
    a.set_state(rho)
    b.set_state(rho)
    m0 = a.mass()
    a.step(1000)
    b.step(1000)
    m1 = a.mass()
    assert np.max(np.abs(m1 / m0 - 1)) < 1e-13
    assert np.array_equal(a.populations(), b.populations())


def test_checkpoint_resume_bitwise():
    w = wl.WORKLOADS["ternary_droplet_2d"].scaled((40, 32))
    announce("checkpoint")
    for prec in ("fp64", "fp32"):
        rho, u = wl.initial_field(w)
        p = F.Params.from_workload(w, precision=prec)
        a = F.Solver(p)
        a.set_state(rho)
        a.step(100)
        blob = a.get_state_raw()
        a.step(50)
        b = F.Solver(p)
        b.set_state_raw(blob)
        assert b.steps == 100
        b.step(50)
        assert np.array_equal(a.populations(), b.populations()), prec


def test_domain_errors():
    w = wl.WORKLOADS["binary_slab_2d"].scaled((16, 4))
    announce("domain errors")
    p = F.Params.from_workload(w)
    s = F.Solver(p)
    rho, _ = wl.initial_field(w)
    bad = rho.copy()
    bad[0, 0, 0, 3] = -1.0
    with pytest.raises(F.FLError) as ei:
        s.set_state(bad)
    assert ei.value.status == F.FL_EDOMAIN
    bad = rho.copy()
    bad[1, 0, 0, 5] = np.nan
    with pytest.raises(F.FLError):
        s.set_state(bad)
    dense = rho.copy() * 3.0        # rho~ b_m >= 1
    with pytest.raises(F.FLError):
        s.set_state(dense)
    s.set_state(rho)
    s.step(5)


def test_numeric_failure_is_reported():
    """A white-noise 3-D ternary field goes unstable (the D3Q19 well-balanced
    scheme's high-wavenumber modes grow); the step reports FL_ENUMERIC."""
    w = wl.WORKLOADS["ternary_droplets_3d"].scaled((24, 16, 16))
    w.noise = 0.05
    announce("numeric failure")
    p = F.Params.from_workload(w, precision="fp64")
    s = F.Solver(p)
    rho, u = wl.initial_field(w)
    s.set_state(rho, u)
    with pytest.raises(F.FLError) as ei:
        s.step(400)
    assert ei.value.status == F.FL_ENUMERIC


def test_run_until_residual():
    w = wl.WORKLOADS["binary_slab_2d"].scaled((32, 2))
    w.noise = 0.0
    announce("run_until")
    p = F.Params.from_workload(w)
    s = F.Solver(p)
    rho, _ = wl.initial_field(w)
    s.set_state(rho)
    conv, done, res = s.run_until(1e-8, 500, 40000)
    print(f"  converged={conv} steps={done} residual={res:.2e}", flush=True)
    assert conv and res < 1e-8 and done % 500 == 0


def test_sampled_timing_steps_like_plain_steps():
    """fl_step_timed_every advances exactly like fl_step (bitwise), times the
    kernels of steps 0, every, 2 every, ... of the call, and rejects every < 1."""
    w = wl.WORKLOADS["binary_slab_3d"].scaled((64, 8, 6))
    announce("sampled timing")
    rho, u = wl.initial_field(w)
    a = F.Solver(F.Params.from_workload(w, precision="fp32"))
    b = F.Solver(F.Params.from_workload(w, precision="fp32"))
    a.set_state(rho, u)
    b.set_state(rho, u)
    kavg, timed = a.step_timed_every(10, 4)
    b.step(10)
    assert timed == 3 and a.steps == b.steps == 10
    assert set(kavg) == {"k_moments_eos", "k_collide_zmarch"} and all(v > 0 for v in kavg.values())
    kavg, timed = a.step_timed_every(600, 1)   # more timed steps than one event pool holds
    b.step(600)
    assert timed == 600
    assert np.array_equal(a.populations(), b.populations())
    with pytest.raises(F.FLError):
        a.step_timed_every(1, 0)
    a.close()
    b.close()


def test_bench_config_full_run_vs_oracle_and_flash():
    """The benchmark configuration at full size over its full run length (D3Q19
    128^3 binary slab, FP32 populations + FP64 EOS, BGK tau 0.8, 20 000 steps,
    default kernels): every (y, z) column identical, the column within 1e-4 of
    the FP64 oracle run of the same problem on 128 x 2 x 2 (the slab is uniform
    along y and z), and the bulk phase errors against the flash equal to the
    oracle's within 1e-3 percentage points."""
    w = wl.WORKLOADS["binary_slab_3d"]
    nx = w.shape[0]
    announce(f"bench configuration {w.shape}, 20000 steps")
    rho, u = wl.initial_field(w)
    s = F.Solver(F.Params.from_workload(w, precision="fp32"))
    s.set_state(rho, u)
    assert list(s.step_timed(1)) == ["k_moments_eos", "k_collide_zmarch"]
    s.step(19999)
    f = s.fields()["rho_molar"].reshape(2, w.shape[2], w.shape[1], nx)
    s.close()
    assert np.array_equal(f, np.broadcast_to(f[:, :1, :1, :], f.shape))
    ws = w.scaled((nx, 2, 2))
    o = oracle_for(ws)
    r2, u2 = wl.initial_field(ws)
    o.init(r2.reshape(2, -1), None if u2 is None else u2.reshape(3, -1))
    o.run(20000)
    ref = o.fields()["rho_molar"].reshape(2, 2, 2, nx)[:, 0, 0, :]
    col = f[:, 0, 0, :]
    err = rel(col, ref)
    mix = mixture_of(w)
    z = ref.sum(axis=1) / ref.sum()
    eg = flash_errors_percent(mix, z, *bulk_values(col))
    eo = flash_errors_percent(mix, z, *bulk_values(ref))
    print(f"  column vs oracle {err:.2e}; errors vs flash (%): GPU {eg}, oracle {eo}", flush=True)
    assert err < 1e-4
    for phase in eg:
        for k in eg[phase]:
            assert abs(eg[phase][k] - eo[phase][k]) < 1e-3, (phase, k)
