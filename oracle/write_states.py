"""Write the thermodynamic inputs of the five synthetic workloads.

TEST INFRASTRUCTURE (calls only ``oracle/``).  Output:
``paper_2212_10680_amd/workload_states.json`` with, per workload, the
components' (Tc, Pc, omega, M, kappa), k_ij, T, and the phase densities of the
flash estimate used to build the initial field (eq. eqInit / eqInit2D):

* lattice units with R = 1 (Sec. IV); the configurations give a_i and b_i, so
  Tc = Ob a/(Oa b R) and Pc = Ob R Tc / b (inverting the PR constants of App. C);
* slab workloads place the liquid with vapor saturation S_V = 0.5, the paper's
  P-x procedure (Sec. IV.B); the pressure is found from the flash;
* droplet workloads use S_L = droplet volume / domain volume;
* the serving workload stores a table of the binary two-phase states along the
  isotherm, parametrised by pressure, from which each request's feed z1
  (drawn at S_V = 0.5) is interpolated.

Run: ``python -m oracle.write_states``.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import thermo as th

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "paper_2212_10680_amd", "workload_states.json")

BIN_A = [2 / 49, 4 / 49]
BIN_B = [2 / 21, 2 / 21]
BIN_W = [0.011, 0.152]
TER_A = [2 / 49, 3 / 49, 4 / 49]
TER_B = [2 / 21, 2 / 21, 2 / 21]
TER_W = [0.011, 0.10, 0.20]
TER_K = [[0.0, 0.02, 0.02], [0.02, 0.0, 0.02], [0.02, 0.02, 0.0]]


def _components(mix, kappa):
    return [{"Tc": float(mix.Tc[i]), "Pc": float(mix.Pc[i]), "omega": float(mix.omega[i]),
             "M": float(mix.M[i]), "kappa": float(kappa[i])} for i in range(mix.n)]


def _state(fr):
    return {"p": float(fr.p), "x": fr.x.tolist(), "y": fr.y.tolist(),
            "rho_L": fr.rho_i_L.tolist(), "rho_V": fr.rho_i_V.tolist(),
            "S_V": float(fr.SV), "beta": float(fr.beta)}


def binary_mixture(kappa):
    return th.lattice_mixture(BIN_A, BIN_B, BIN_W, 1, 0.8, kappa=kappa)


def ternary_mixture(kappa):
    return th.lattice_mixture(TER_A, TER_B, TER_W, 2, 0.85, kij=np.array(TER_K), kappa=kappa)


def binary_isotherm_table(mix, npts=240):
    """Two-phase binary states along the isotherm, as functions of pressure."""
    rows = []
    ps = np.linspace(0.0256, 0.1755, npts)
    for p in ps:
        # binary: phase compositions depend on p only; flash a feed between them
        for z1 in (0.3, 0.1, 0.45, 0.02, 0.55):
            fr = th.flash(mix, [z1, 1 - z1], p)
            if fr.two_phase:
                break
        if not fr.two_phase:
            continue
        vL, vV = fr.vL, fr.vV
        beta_half = vL / (vL + vV)     # S_V = 0.5
        z1_half = beta_half * fr.y[0] + (1 - beta_half) * fr.x[0]
        rows.append({"p": float(p), "x1": float(fr.x[0]), "y1": float(fr.y[0]),
                     "rho_L": fr.rho_i_L.tolist(), "rho_V": fr.rho_i_V.tolist(),
                     "z1_at_SV_half": float(z1_half)})
    return rows


def e1_state(eos):
    Tc, Pc, om, M, sT, sP = th.physical_to_lattice(["C3", "nC5"], eos)
    kappa = [0.10, 0.15]
    mix = th.Mixture(Tc, Pc, om, 370.03 * sT, eos=eos, R=1.0, M=M, kappa=np.array(kappa))
    z = [0.4, 0.6]
    fr = th.flash(mix, z, 16.547 * sP)
    comps = [{"Tc": float(Tc[i]), "Pc": float(Pc[i]), "omega": float(om[i]), "M": float(M[i]),
              "kappa": kappa[i]} for i in range(2)]
    return {"components": comps, "kij": np.zeros((2, 2)).tolist(), "T": float(mix.T), "z": z,
            "eos": eos, "T_scale_per_K": sT, "p_scale_per_bar": sP, "state": _state(fr)}


def e5_state():
    """Sec. IV.C: C1/C2/C3, z = (0.4, 0.3, 0.3), PR, 216.483 K, 20.684 bar."""
    Tc, Pc, om, M, sT, sP = th.physical_to_lattice(["C1", "C2", "C3"], "PR")
    kappa = [0.05, 0.10, 0.15]
    mix = th.Mixture(Tc, Pc, om, 216.483 * sT, eos="PR", R=1.0, M=M, kappa=np.array(kappa))
    z = [0.4, 0.3, 0.3]
    fr = th.flash(mix, z, 20.684 * sP)
    comps = [{"Tc": float(Tc[i]), "Pc": float(Pc[i]), "omega": float(om[i]), "M": float(M[i]),
              "kappa": kappa[i]} for i in range(3)]
    return {"components": comps, "kij": np.zeros((3, 3)).tolist(), "T": float(mix.T), "z": z,
            "eos": "PR", "T_scale_per_K": sT, "p_scale_per_bar": sP, "state": _state(fr)}


def e6_state():
    """Sec. IV.D: C2/nC5 at 387.70 K, uniform x = (0.62, 0.38) at the molar
    density whose EOS pressure is 50 bar (the one real root)."""
    Tc, Pc, om, M, sT, sP = th.physical_to_lattice(["C2", "nC5"], "PR")
    kappa = [0.10, 0.15]
    mix = th.Mixture(Tc, Pc, om, 387.70 * sT, eos="PR", R=1.0, M=M, kappa=np.array(kappa))
    x = np.array([0.62, 0.38])
    roots = mix.volume_roots(50.0 * sP, x)
    assert len(roots) == 1
    rho = x / roots[0]
    comps = [{"Tc": float(Tc[i]), "Pc": float(Pc[i]), "omega": float(om[i]), "M": float(M[i]),
              "kappa": kappa[i]} for i in range(2)]
    return {"components": comps, "kij": np.zeros((2, 2)).tolist(), "T": float(mix.T), "z": x.tolist(),
            "eos": "PR", "T_scale_per_K": sT, "p_scale_per_bar": sP,
            "state": {"p": float(mix.pressure(rho)), "rho_uniform": rho.tolist()}}


def e7_state():
    """Sec. IV.E: C3/nC5 flash with PR at 340 K and 5 bar (density ratio
    50.97); the phase compositions do not depend on the feed inside the
    two-phase region, so the feed is z = (0.5, 0.5)."""
    Tc, Pc, om, M, sT, sP = th.physical_to_lattice(["C3", "nC5"], "PR")
    kappa = [0.05, 0.10]
    mix = th.Mixture(Tc, Pc, om, 340.0 * sT, eos="PR", R=1.0, M=M, kappa=np.array(kappa))
    fr = th.flash(mix, [0.5, 0.5], 5.0 * sP)
    comps = [{"Tc": float(Tc[i]), "Pc": float(Pc[i]), "omega": float(om[i]), "M": float(M[i]),
              "kappa": kappa[i]} for i in range(2)]
    return {"components": comps, "kij": np.zeros((2, 2)).tolist(), "T": float(mix.T), "z": [0.5, 0.5],
            "eos": "PR", "T_scale_per_K": sT, "p_scale_per_bar": sP, "state": _state(fr)}


def envelope_states():
    """Sec. IV.B: C2/nC5 with PR; p-x points on the isotherms 274.96 K and
    387.70 K, T-x points on the isobars 30, 45 and 58 bar, each at the feed
    that gives S_V = 0.5 (the phase compositions of a binary at fixed T and p
    do not depend on the feed)."""
    Tc, Pc, om, M, sT, sP = th.physical_to_lattice(["C2", "nC5"], "PR")
    kappa = [0.1, 0.2]

    def point(T_K, p_bar):
        mix = th.Mixture(Tc, Pc, om, T_K * sT, eos="PR", R=1.0, M=M, kappa=np.array(kappa))
        for z1 in np.linspace(0.02, 0.98, 49):
            fr = th.flash(mix, [z1, 1 - z1], p_bar * sP)
            if fr.two_phase:
                break
        assert fr.two_phase, (T_K, p_bar)
        beta = fr.vL / (fr.vL + fr.vV)          # vapor mole fraction at S_V = 0.5
        z1 = beta * fr.y[0] + (1 - beta) * fr.x[0]
        return {"T_K": T_K, "p_bar": p_bar, "T": float(mix.T), "p": float(fr.p), "x1": float(fr.x[0]),
                "y1": float(fr.y[0]), "z1": float(z1), "rho_L": fr.rho_i_L.tolist(), "rho_V": fr.rho_i_V.tolist()}

    curves = [
        {"kind": "isotherm", "T_K": 274.96, "points": [point(274.96, p) for p in (4.0, 8.0, 12.0, 16.0, 20.0, 23.0)]},
        {"kind": "isotherm", "T_K": 387.70, "points": [point(387.70, p) for p in (10.0, 20.0, 30.0, 40.0, 50.0, 60.0)]},
        {"kind": "isobar", "p_bar": 30.0, "points": [point(T, 30.0) for T in (290.0, 325.0, 360.0, 395.0, 430.0, 455.0)]},
        {"kind": "isobar", "p_bar": 45.0, "points": [point(T, 45.0) for T in (310.0, 340.0, 370.0, 400.0, 430.0, 448.0)]},
        {"kind": "isobar", "p_bar": 58.0, "points": [point(T, 58.0) for T in (330.0, 350.0, 370.0, 390.0, 410.0, 422.0)]},
    ]
    comps = [{"Tc": float(Tc[i]), "Pc": float(Pc[i]), "omega": float(om[i]), "M": float(M[i]),
              "kappa": kappa[i]} for i in range(2)]
    return {"components": comps, "kij": np.zeros((2, 2)).tolist(), "eos": "PR", "T_scale_per_K": sT,
            "p_scale_per_bar": sP, "curves": curves}


def main():
    out = {"_note": "written by oracle/write_states.py; lattice units, R = 1"}
    # binary, T = 0.8 Tc2; z1 = 0.3 at S_V = 0.5 (the literal z1 = 0.5 has no
    # S_V = 0.5 two-phase state on this isotherm)
    kap_bin = [0.10, 0.15]
    mix = binary_mixture(kap_bin)
    p, fr = th.pressure_for_saturation(mix, [0.3, 0.7], 0.5, 0.03, 0.18)
    out["binary_z03"] = {"components": _components(mix, kap_bin), "kij": np.zeros((2, 2)).tolist(),
                         "T": float(mix.T), "z": [0.3, 0.7], "state": _state(fr)}
    # ternary, T = 0.85 Tc3, z = (0.2, 0.3, 0.5) (the literal (0.5, 0.3, 0.2) is
    # single phase at this T)
    kap_ter = [0.05, 0.10, 0.15]
    tmix = ternary_mixture(kap_ter)
    z = [0.2, 0.3, 0.5]
    SL1 = math.pi * 40.0**2 / 256.0**2
    p1, fr1 = th.pressure_for_saturation(tmix, z, 1.0 - SL1, 0.02, 0.16)
    SL4 = 2.0 * (4.0 / 3.0) * math.pi * 30.0**3 / 256.0**3
    p4, fr4 = th.pressure_for_saturation(tmix, z, 1.0 - SL4, 0.02, 0.16)
    out["ternary_droplet2d"] = {"components": _components(tmix, kap_ter), "kij": TER_K,
                                "T": float(tmix.T), "z": z, "S_L": SL1, "state": _state(fr1)}
    out["ternary_droplets3d"] = {"components": _components(tmix, kap_ter), "kij": TER_K,
                                 "T": float(tmix.T), "z": z, "S_L": SL4, "state": _state(fr4)}
    out["binary_isotherm"] = {"components": _components(mix, kap_bin), "kij": np.zeros((2, 2)).tolist(),
                              "T": float(mix.T), "table": binary_isotherm_table(mix)}
    # the paper's case of Sec. IV.A: C3/nC5, z = (0.4, 0.6), T = 370.03 K,
    # p = 16.547 bar, PR and SRK, kappa = (0.10, 0.15), in lattice units by the
    # conversion rule of Sec. IV
    for eos in ("PR", "SRK"):
        out["e1_c3c5_" + eos] = e1_state(eos)
    out["e5_c1c2c3"] = e5_state()
    out["e6_c2c5_spinodal"] = e6_state()
    out["e7_c3c5_droplet"] = e7_state()
    out["e2e3_c2c5_envelopes"] = envelope_states()
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
