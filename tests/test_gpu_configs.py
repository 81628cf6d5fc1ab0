"""The synthetic workloads at their own sizes and run lengths, GPU against the
FP64 oracle, through the C ABI.

* binary_slab_2d (D2Q9 64x8, two PR components, tanh slab with +-1 % seeded
  noise, BGK tau = 1, FP64, 20 000 steps): element by element against the
  oracle run of the same length; the chemical potential mu_i = RT ln f_i +
  mu_I,i (Sec. III.B steps 5-6) constant on each even/odd sublattice (the
  discrete form of equal fugacities, R-18: central differences cannot see the
  sublattice modes the noise seeds); bulk phases against a flash at the LBM's
  bulk pressure (the comparison of Sec. IV.A), GPU errors equal to the
  oracle's.
* ternary_droplet_2d (D2Q9 256^2, three components, droplet of radius 40,
  MRT tau = 1, 50 000 steps), FP64 and FP32 populations: the central row and
  column, the pressure jump across the interface and the per-component mass
  against the oracle's values at steps 1 000 and 50 000
  (tests/golden/config_goldens.json, written by write_config_goldens.py from
  oracle/ alone), and the Young-Laplace check of Sec. V: (p_in - p_out) R
  against sigma of eq. eqMCsigma.
* ternary_droplets_3d at 64^3 (the 256^3 two-droplet workload scaled by 1/4,
  MRT tau = 0.8, isotropic stencils), FP32 populations as in the benchmark and
  FP64: the line through both droplet centres and the line across the neck at
  steps 100 and 1 000, and the per-component mass drift.
"""
import json
import os

import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import workloads as wl

from _util import bulk_values, flash_errors_percent, mixture_of, oracle_for, rel

pytestmark = pytest.mark.gpu

GOLDEN_PATH = os.path.join(os.path.dirname(__file__), "golden", "config_goldens.json")


def golden(name):
    with open(GOLDEN_PATH) as f:
        return json.load(f)[name]


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def mu_fields(mix, rt, lnf, shape):
    """mu_i = RT ln f_i - sum_j kappa_ij lap(rho~_j) with the axis stencils
    (eqs. eqChemPotI2, eqkappa, eq2ndder) on a periodic D2Q9 lattice."""
    nx, ny = shape
    r = rt.reshape(-1, ny, nx)
    lap = (np.roll(r, 1, 2) + np.roll(r, -1, 2) + np.roll(r, 1, 1) + np.roll(r, -1, 1) - 4 * r)
    kij = np.sqrt(np.outer(mix.kappa, mix.kappa))
    return mix.RT * lnf.reshape(-1, ny, nx) - np.einsum("ij,jyx->iyx", kij, lap)


def sublattice_spread(mu):
    """Largest spread (max - min) of mu_i over one (x, y) parity sublattice."""
    return max(float(np.ptp(mu[i, yp::2, xp::2])) for i in range(mu.shape[0]) for yp in (0, 1) for xp in (0, 1))


def test_binary_slab_2d_full_run():
    w = wl.WORKLOADS["binary_slab_2d"]
    nx, ny = w.shape
    announce(f"binary_slab_2d {w.shape}, {w.steps} steps, FP64")
    rho, _ = wl.initial_field(w)
    o = oracle_for(w)
    o.init(rho.reshape(w.ncomp, -1))
    s = F.Solver(F.Params.from_workload(w))
    s.set_state(rho)
    o.run(w.steps)
    s.step(w.steps)
    fo, fs = o.fields(), s.fields()
    s.close()
    er, el, ep = (rel(fs[k], fo[k]) for k in ("rho_molar", "lnf", "p"))
    eu = float(np.max(np.abs(fs["u"] - fo["u"])))
    print(f"  after {w.steps} steps: rho {er:.1e} lnf {el:.1e} p {ep:.1e} |du| {eu:.1e} "
          f"(|u|max {np.abs(fo['u']).max():.1e})", flush=True)
    assert er < 1e-10 and el < 1e-10 and ep < 1e-10 and eu < 1e-12
    mix = mixture_of(w)
    sg = sublattice_spread(mu_fields(mix, fs["rho_molar"], fs["lnf"], w.shape))
    so = sublattice_spread(mu_fields(mix, fo["rho_molar"], fo["lnf"], w.shape))
    print(f"  mu_i spread on a parity sublattice: GPU {sg:.2e}, oracle {so:.2e}", flush=True)
    assert sg < 1e-5 and abs(sg - so) < 1e-9
    # bulk phases (rows averaged: an even number of them) against the flash
    row = lambda f: f["rho_molar"].reshape(w.ncomp, ny, nx).mean(axis=1)
    z = row(fs).sum(axis=1) / row(fs).sum()
    eg = flash_errors_percent(mix, z, *bulk_values(row(fs)), names=("1", "2"))
    eo = flash_errors_percent(mix, z, *bulk_values(row(fo)), names=("1", "2"))
    print(f"  errors vs flash at the bulk pressure (%): GPU {eg}", flush=True)
    for ph in eg:
        for k in eg[ph]:
            assert abs(eg[ph][k] - eo[ph][k]) < 1e-7, (ph, k, eg[ph][k], eo[ph][k])


def _droplet_run(w, precision, stops):
    rho, _ = wl.initial_field(w)
    s = F.Solver(F.Params.from_workload(w, precision=precision))
    s.set_state(rho)
    m0 = s.mass()
    out = {}
    for n in stops:
        s.step(n - s.steps)
        f = s.fields()
        out[n] = (f, s.mass())
    s.close()
    return m0, out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ternary_droplet_2d_full_run(precision):
    w = wl.WORKLOADS["ternary_droplet_2d"]
    nx, ny = w.shape
    g = golden("droplet2d")
    announce(f"ternary_droplet_2d {w.shape}, {w.steps} steps, {precision}")
    m0, out = _droplet_run(w, precision, (1000, w.steps))
    # FP64: element by element after 1 000 steps; after 50 000 the droplet is
    # at rest but a rounding-seeded drift of the interface (a neutral mode:
    # translation costs nothing) leaves ~1e-8 between trajectories there, so the
    # comparison is on translation-invariant bulk values (R-18), with the
    # element-wise difference reported.  FP32: 1e-4 throughout.
    bar = {1000: 1e-10, w.steps: 1e-6} if precision == "fp64" else {1000: 1e-4, w.steps: 1e-4}
    mix = mixture_of(w)
    rL, rV, _ = w.phase_densities()
    level = 0.5 * (float(np.sum(rL)) + float(np.sum(rV)))
    for n, (f, mass) in out.items():
        ref = g["checkpoints"][str(n)]
        r = f["rho_molar"].reshape(w.ncomp, ny, nx)
        p = f["p"].reshape(ny, nx)
        c = nx // 2
        e_row = rel(r[:, ny // 2, :], np.array(ref["row_rho"]))
        e_col = rel(r[:, :, c], np.array(ref["col_rho"]))
        e_p = rel(p[ny // 2, :], np.array(ref["row_p"]))
        dp = float(p[c - 1:c + 1, c - 1:c + 1].mean() - p[0:2, 0:2].mean())
        dp_ref = ref["p_in"] - ref["p_out"]
        R = float(np.sqrt(np.count_nonzero(r.sum(axis=0) > level) / np.pi))
        e_m = float(np.max(np.abs(mass / np.array(ref["mass"]) - 1)))
        print(f"  step {n}: row {e_row:.1e} col {e_col:.1e} p {e_p:.1e} mass {e_m:.1e}; dp {dp:.6e} "
              f"(oracle {dp_ref:.6e}, rel {abs(dp / dp_ref - 1):.1e}); R {R:.3f} (oracle {ref['radius']:.3f})",
              flush=True)
        assert e_row < bar[n] and e_col < bar[n] and e_p < bar[n]
        # bulk values: the central 8 nodes of the row (droplet core) and the 8
        # nodes around the periodic edge of the row (vapour)
        core = lambda rr: rr[:, c - 4:c + 4].mean(axis=1)
        vap = lambda rr: np.concatenate([rr[:, :4], rr[:, -4:]], axis=1).mean(axis=1)
        rr, rf = r[:, ny // 2, :], np.array(ref["row_rho"])
        e_bulk = max(rel(core(rr), core(rf)), rel(vap(rr), vap(rf)))
        print(f"    bulk core/vapour vs oracle {e_bulk:.1e}", flush=True)
        assert e_bulk < (1e-9 if precision == "fp64" else 1e-4)
        assert abs(dp / dp_ref - 1) < (1e-4 if precision == "fp64" else 1e-3)
        # R counts the nodes above the mid-density: in FP32 one node at the
        # threshold may fall on the other side (R changes by ~1 / (2 pi R))
        assert abs(R - ref["radius"]) < (1e-9 if precision == "fp64" else 0.01)
        assert e_m < (1e-12 if precision == "fp64" else 1e-6)
    drift = float(np.max(np.abs(out[w.steps][1] / m0 - 1)))
    sigma = g["sigma_flat"]
    f, _ = out[w.steps]
    print(f"  mass drift over {w.steps} steps {drift:.1e}; Young-Laplace (p_in - p_out) R / sigma = "
          f"{dp * R / sigma:.4f} (sigma {sigma:.5f})", flush=True)
    assert drift < (1e-12 if precision == "fp64" else 1e-6)
    # the Laplace law holds to O(W / R) (interface width 4, radius 40)
    assert abs(dp * R / sigma - 1) < 0.1


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_ternary_droplets_3d_at_64_vs_oracle(precision):
    w = wl.WORKLOADS["ternary_droplets_3d"].scaled((64, 64, 64))
    g = golden("droplets3d")
    assert g["shape"] == list(w.shape) and abs(g["radius"] - w.radius) < 1e-12
    n = 64
    announce(f"ternary_droplets_3d at {w.shape}, isotropic stencils, {precision}")
    rho, u = wl.initial_field(w)
    s = F.Solver(F.Params.from_workload(w, precision=precision, stencil="isotropic"))
    s.set_state(rho, u)
    m0 = s.mass()
    # u_x (absolute; the approach speed is 0.02) to 5e-4 of it in FP32 and
    # 5e-9 in FP64
    bar, ubar = (1e-4, 1e-5) if precision == "fp32" else (1e-10, 1e-10)
    for stop in (100, 1000):
        s.step(stop - s.steps)
        f = s.fields()
        ref = g["checkpoints"][str(stop)]
        r = f["rho_molar"].reshape(w.ncomp, n, n, n)
        ux = f["u"].reshape(3, n, n, n)[0]
        c = n // 2
        e_ax = rel(r[:, c, c, :], np.array(ref["axis_rho"]))
        e_nk = rel(r[:, c, :, c], np.array(ref["neck_rho"]))
        e_u = float(np.max(np.abs(ux[c, c, :] - np.array(ref["axis_ux"]))))
        e_m = float(np.max(np.abs(s.mass() / np.array(ref["mass"]) - 1)))
        print(f"  step {stop}: axis {e_ax:.1e} neck {e_nk:.1e} |du_x| {e_u:.1e} mass {e_m:.1e}", flush=True)
        assert e_ax < bar and e_nk < bar and e_u < ubar
        assert e_m < (1e-12 if precision == "fp64" else 1e-6)
    drift = np.abs(s.mass() / m0 - 1)
    print(f"  per-component mass drift over 1000 steps: {drift}", flush=True)
    assert np.all(drift < (1e-12 if precision == "fp64" else 1e-7))
    s.close()
