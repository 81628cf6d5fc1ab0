"""Writes the FP64 oracle's reference values for the full-length workload runs
(tests/golden/config_goldens.json).  Calls only oracle/ (and the seeded input
generators of the package, which hold none of the method's arithmetic).

* ternary_droplet_2d: D2Q9 256^2, three PR components, a static droplet of
  radius 40 (eq. eqInit2D, h = 1), MRT tau = 1, FP64, 50 000 steps.  Stored at
  steps 1 000 and 50 000: the central row and column of the molar densities and
  the pressure along the row, the per-component mass, the pressure jump
  p_in - p_out between the droplet centre and the far corner, the droplet
  radius from the area inside the mid-density contour, and the interfacial
  tension of eq. eqMCsigma from the discrete flat-interface equilibrium of the
  same mixture (Newton), for the Young-Laplace comparison of Sec. V.
* ternary_droplets_3d at 64^3: the 256^3 two-droplet workload scaled by 1/4
  (radius 7.5, centres 17.5 apart, approaching at +-0.02), MRT tau = 0.8,
  isotropic stencils, 1 000 steps.  Stored at steps 100 and 1 000: the line
  through both droplet centres (densities and u_x), the line across the neck
  along y, and the per-component mass.

Usage: python tests/golden/write_config_goldens.py [droplet2d] [droplets3d]
(both by default).  Takes about 40 + 10 minutes on 8 cores.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fixed_point as fp  # noqa: E402
from oracle import lbm  # noqa: E402
from oracle import thermo as th  # noqa: E402
from paper_2212_10680_amd import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "config_goldens.json")


def mixture(w):
    comps, kij, T = w.thermo()
    return th.Mixture([c["Tc"] for c in comps], [c["Pc"] for c in comps], [c["omega"] for c in comps],
                      T, kij=kij, M=[c["M"] for c in comps], kappa=[c["kappa"] for c in comps])


def droplet_radius(tot, rL, rV):
    """Radius of the region where the total molar density exceeds the
    mid-density (rL + rV) / 2, from its area (2-D)."""
    return float(np.sqrt(np.count_nonzero(tot > 0.5 * (rL + rV)) / np.pi))


def flat_sigma(mix, w):
    """eq. eqMCsigma on the discrete flat-interface equilibrium of the mixture
    at the droplet state (1-D slab of 200 nodes, Newton)."""
    rL, rV, _ = w.phase_densities()
    n = 200
    x = np.arange(n, dtype=np.float64)
    slab = np.stack([wl.slab_profile(x, n, rL[i], rV[i], 0.5, w.W) for i in range(len(rL))])
    rho, lam, res = fp.solve(mix, slab, mix.kappa)
    return fp.interfacial_tension(mix, rho, mix.kappa), float(res)


def droplet2d():
    w = wl.WORKLOADS["ternary_droplet_2d"]
    mix = mixture(w)
    nx, ny = w.shape
    rho, _ = wl.initial_field(w)
    o = lbm.OracleLBM(mix, w.lattice, w.shape, tau=w.tau, collision=w.collision)
    o.init(rho.reshape(w.ncomp, -1))
    rL, rV, _ = w.phase_densities()
    out = {"workload": w.name, "shape": list(w.shape), "collision": w.collision, "tau": w.tau,
           "checkpoints": {}}
    sigma, res = flat_sigma(mix, w)
    out["sigma_flat"] = sigma
    out["sigma_newton_residual"] = res
    t0 = time.time()
    for target in (1000, 50000):
        o.run(target - o.steps)
        f = o.fields()
        r = f["rho_molar"].reshape(w.ncomp, ny, nx)
        p = f["p"].reshape(ny, nx)
        tot = r.sum(axis=0)
        c = nx // 2
        out["checkpoints"][str(target)] = {
            "row_rho": r[:, ny // 2, :].tolist(),
            "col_rho": r[:, :, c].tolist(),
            "row_p": p[ny // 2, :].tolist(),
            "mass": o.mass().tolist(),
            "p_in": float(p[c - 1:c + 1, c - 1:c + 1].mean()),
            "p_out": float(p[0:2, 0:2].mean()),
            "radius": droplet_radius(tot, float(np.sum(rL)), float(np.sum(rV))),
            "u_max": float(np.abs(f["u"]).max()),
        }
        print(f"droplet2d step {o.steps} ({time.time() - t0:.0f} s)", flush=True)
    return out


def droplets3d():
    w = wl.WORKLOADS["ternary_droplets_3d"].scaled((64, 64, 64))
    mix = mixture(w)
    n = 64
    rho, u = wl.initial_field(w)
    o = lbm.OracleLBM(mix, w.lattice, w.shape, tau=w.tau, collision=w.collision, stencil="isotropic")
    o.init(rho.reshape(w.ncomp, -1), u.reshape(w.D, -1))
    out = {"workload": w.name, "shape": list(w.shape), "radius": w.radius, "separation": w.separation,
           "u0": w.u0, "stencil": "isotropic", "checkpoints": {}}
    t0 = time.time()
    for target in (100, 1000):
        o.run(target - o.steps)
        f = o.fields()
        r = f["rho_molar"].reshape(w.ncomp, n, n, n)
        ux = f["u"].reshape(w.D, n, n, n)[0]
        c = n // 2
        out["checkpoints"][str(target)] = {
            "axis_rho": r[:, c, c, :].tolist(),     # along x through both centres
            "axis_ux": ux[c, c, :].tolist(),
            "neck_rho": r[:, c, :, c].tolist(),     # along y through the midpoint
            "mass": o.mass().tolist(),
        }
        print(f"droplets3d step {o.steps} ({time.time() - t0:.0f} s)", flush=True)
    return out


def main():
    which = sys.argv[1:] or ["droplets3d", "droplet2d"]
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in which:
        data[name] = {"droplet2d": droplet2d, "droplets3d": droplets3d}[name]()
        with open(OUT, "w") as f:
            json.dump(data, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
