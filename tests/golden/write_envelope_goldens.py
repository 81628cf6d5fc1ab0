"""Writes the FP64 oracle's states for the p-x and T-x envelope points of
Sec. IV.B (tests/golden/envelope_goldens.json).  Calls only oracle/ (and the
package's seeded input generators, which hold none of the method's
arithmetic).

Each point: C2/nC5 (PR), D2Q9 200 x 2, BGK tau = 1.25, kappa = (0.1, 0.2), the
eq. eqInit slab at S_V = 0.5 with W = 4, 5e5 steps (the paper's run length).
Stored per point, after 1e5 and after 5e5 steps: the molar densities of one
row (the lattice is uniform along y), the net momentum sum_x rho u_x and the
largest |u|.  At some points the centred slab is unstable to translation (its
net momentum grows from rounding), so later states depend on rounding: the
1e5-step checkpoint comes before that growth is visible.

Usage: python tests/golden/write_envelope_goldens.py [processes]  (default 8;
one oracle thread per process).  About 15 minutes on 8 cores.
"""
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "envelope_goldens.json")


def _init():
    from oracle import lbm
    lbm.set_threads(1)


def run_point(job):
    from oracle import lbm
    from oracle import thermo as th
    from paper_2212_10680_amd import workloads as wl

    ci, k = job
    comps, curves = wl.envelope_curves()
    pt = curves[ci]["points"][k]
    E = wl.ENVELOPE
    mix = th.Mixture([c["Tc"] for c in comps], [c["Pc"] for c in comps], [c["omega"] for c in comps],
                     pt["T"], eos="PR", R=1.0, M=[c["M"] for c in comps], kappa=[c["kappa"] for c in comps])
    o = lbm.OracleLBM(mix, "D2Q9", E["shape"], tau=E["tau"])
    o.init(wl.envelope_field(pt).reshape(2, -1))
    t0 = time.time()
    nx, ny = E["shape"]
    out = {}
    for stop in (100000, E["steps"]):
        o.run(stop - o.steps)
        f = o.fields()
        r = f["rho_molar"].reshape(2, ny, nx)
        ux = f["u"].reshape(2, ny, nx)[0]
        mom = float(np.sum(np.einsum("i,iyx->yx", mix.M, r) * ux))
        out[str(stop)] = {"row": r[:, 0, :].tolist(), "momentum": mom, "u_max": float(np.abs(f["u"]).max())}
    return ci, k, out, time.time() - t0


def main():
    from paper_2212_10680_amd import workloads as wl

    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    _, curves = wl.envelope_curves()
    jobs = [(ci, k) for ci, c in enumerate(curves) for k in range(len(c["points"]))]
    out = {"steps": wl.ENVELOPE["steps"], "shape": list(wl.ENVELOPE["shape"]), "tau": wl.ENVELOPE["tau"],
           "curves": [[None] * len(c["points"]) for c in curves]}
    with Pool(procs, initializer=_init) as pool:
        for ci, k, rec, dt in pool.imap_unordered(run_point, jobs):
            out["curves"][ci][k] = rec
            print(f"curve {ci} point {k}: {dt:.0f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
