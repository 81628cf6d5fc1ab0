"""Synthetic workloads and their seeded initial fields.

This module holds no step of the lattice update and no thermodynamics: it only
* names the five workloads (lattice, shape, relaxation, precision form),
* reads their thermodynamic inputs (component constants, temperature, flash
  phase densities) from ``workload_states.json``, which the oracle's state
  writer produced, and
* builds initial molar-density fields with the paper's geometry recipes: the
  tanh slab of eq. ``eqInit`` (Sec. IV.A), the tanh droplet of
  eq. ``eqInit2D`` (Sec. IV.E, h = 1 for a circle, extended to a sphere in 3-D),
  a uniform state (Sec. IV.D), plus seeded multiplicative noise (numpy PCG64).

Both the GPU path and the oracle are fed from here, so they see identical bits.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
STATES_PATH = os.path.join(HERE, "workload_states.json")

_states = None


def states():
    global _states
    if _states is None:
        with open(STATES_PATH) as f:
            _states = json.load(f)
    return _states


@dataclass
class Workload:
    name: str
    lattice: str                 # "D2Q9" | "D3Q19"
    shape: tuple                 # (nx, ny) or (nx, ny, nz)
    collision: str               # "BGK" | "MRT"
    tau: float
    precision: str               # "fp64" | "fp32"
    steps: int
    state_key: str
    geometry: str                # "slab" | "droplet" | "two_droplets"
    ncomp: int
    kappa_scale: float = 0.5
    W: float = 4.0
    SV: float | None = 0.5       # None: the flash state's vapor saturation
    radius: float = 0.0
    h: float = 1.0               # y semi-axis / x semi-axis of a droplet (eqInit2D)
    separation: float = 0.0
    u0: float = 0.0
    noise: float = 0.0
    seed: int = 0
    eos: str = "PR"
    extra: dict = field(default_factory=dict)

    @property
    def D(self):
        return 2 if self.lattice == "D2Q9" else 3

    @property
    def nodes(self):
        return int(np.prod(self.shape))

    def thermo(self):
        """Component list (Tc, Pc, omega, M, kappa), k_ij and T, lattice units."""
        st = states()[self.state_key]
        comps = [dict(c) for c in st["components"]]
        for c in comps:
            c["kappa"] *= self.kappa_scale
        return comps, np.array(st["kij"], dtype=np.float64), float(st["T"])

    @property
    def vapor_saturation(self):
        return self.SV if self.SV is not None else float(states()[self.state_key]["state"]["S_V"])

    def phase_densities(self):
        st = states()[self.state_key]["state"]
        return np.array(st["rho_L"]), np.array(st["rho_V"]), float(st["p"])

    def scaled(self, shape):
        """Same workload on another lattice shape, geometry scaled with nx."""
        f = shape[0] / self.shape[0]
        w = Workload(**{**self.__dict__, "extra": dict(self.extra)})
        w.shape = tuple(shape)
        w.radius = self.radius * f
        w.separation = self.separation * f
        return w


WORKLOADS = {
    # D2Q9 64x8 periodic binary slab, BGK tau = 1, FP64, +-1 % noise
    "binary_slab_2d": Workload("binary_slab_2d", "D2Q9", (64, 8), "BGK", 1.0, "fp64", 20000,
                               "binary_z03", "slab", 2, noise=0.01),
    # D2Q9 256^2 ternary static droplet R = 40, MRT
    "ternary_droplet_2d": Workload("ternary_droplet_2d", "D2Q9", (256, 256), "MRT", 1.0, "fp64",
                                   50000, "ternary_droplet2d", "droplet", 3, radius=40.0),
    # D3Q19 128^3 binary slab, BGK tau = 0.8, FP32 populations + FP64 EOS
    "binary_slab_3d": Workload("binary_slab_3d", "D3Q19", (128, 128, 128), "BGK", 0.8, "fp32",
                               20000, "binary_z03", "slab", 2),
    # 512 binary D2Q9 L x 8 slabs (per-request parameters drawn elsewhere)
    "serving_binary_2d": Workload("serving_binary_2d", "D2Q9", (64, 8), "BGK", 1.0, "fp32",
                                  0, "binary_isotherm", "slab", 2),
    # D3Q19 256^3 ternary, two droplets R = 30, centres 70 apart, +-0.02 approach
    "ternary_droplets_3d": Workload("ternary_droplets_3d", "D3Q19", (256, 256, 256), "MRT", 0.8,
                                    "fp32", 20000, "ternary_droplets3d", "two_droplets", 3,
                                    radius=30.0, separation=70.0, u0=0.02),
    # the paper's flat-interface case of Sec. IV.A: C3/nC5 (z = 0.4/0.6) at
    # 370.03 K and 16.547 bar, D2Q9 400 x 2, tau = 0.8, kappa = (0.10, 0.15)
    # as given, W = 8, S_V from the flash, 1e6 steps; PR and SRK
    "e1_c3c5_pr": Workload("e1_c3c5_pr", "D2Q9", (400, 2), "BGK", 0.8, "fp64", 1000000,
                           "e1_c3c5_PR", "slab", 2, kappa_scale=1.0, W=8.0, SV=None, eos="PR"),
    "e1_c3c5_srk": Workload("e1_c3c5_srk", "D2Q9", (400, 2), "BGK", 0.8, "fp64", 1000000,
                            "e1_c3c5_SRK", "slab", 2, kappa_scale=1.0, W=8.0, SV=None, eos="SRK"),
    # Sec. IV.C: C1/C2/C3 (z = 0.4/0.3/0.3) at 216.483 K and 20.684 bar, D2Q9
    # 200 x 2, tau = 1, kappa = (0.05, 0.10, 0.15), W = 4, S_V from the flash
    "e5_c1c2c3": Workload("e5_c1c2c3", "D2Q9", (200, 2), "BGK", 1.0, "fp64", 1000000,
                          "e5_c1c2c3", "slab", 3, kappa_scale=1.0, W=4.0, SV=None),
    # Sec. IV.E: elliptical C3/nC5 droplet (R0 = 30, h = 0.9, W = 4) in PR at
    # 340 K and 5 bar (density ratio 50.97), D2Q9 200 x 200, tau = 0.85,
    # kappa = (0.05, 0.10), 4000 steps
    "e7_droplet": Workload("e7_droplet", "D2Q9", (200, 200), "BGK", 0.85, "fp64", 4000,
                           "e7_c3c5_droplet", "droplet", 2, kappa_scale=1.0, radius=30.0, h=0.9),
    # Sec. IV.D: C2/nC5 spinodal decomposition from a uniform x = (0.62, 0.38)
    # at 50 bar and 387.70 K, D2Q9 200 x 200, tau = 1.15, kappa = (0.10, 0.15);
    # +-1 % seeded fluctuation of the total density (amplitude not given)
    "e6_spinodal": Workload("e6_spinodal", "D2Q9", (200, 200), "BGK", 1.15, "fp64", 500000,
                            "e6_c2c5_spinodal", "uniform", 2, kappa_scale=1.0, noise=0.01),
}


# Sec. IV.B p-x and T-x envelopes: C2/nC5 (PR), D2Q9 200 x 2, tau = 1.25,
# kappa = (0.1, 0.2), W = 4, S_V = 0.5, 5e5 steps per point; the points (T, p
# and flash phase densities) are in the states file
ENVELOPE = dict(state_key="e2e3_c2c5_envelopes", shape=(200, 2), tau=1.25, W=4.0, SV=0.5, steps=500000)


def envelope_curves():
    """(components, curves): the curves' points with T, p (lattice units and
    K, bar) and the flash phase densities."""
    st = states()[ENVELOPE["state_key"]]
    return [dict(c) for c in st["components"]], st["curves"]


def envelope_field(point):
    """eq. eqInit slab of one envelope point, [2, 1, ny, nx]."""
    nx, ny = ENVELOPE["shape"]
    x = np.broadcast_to(np.arange(nx, dtype=np.float64), (1, ny, nx))
    return np.ascontiguousarray(np.stack([slab_profile(x, nx, point["rho_L"][i], point["rho_V"][i],
                                                       ENVELOPE["SV"], ENVELOPE["W"]) for i in range(2)]))


def _grid(shape):
    """Node coordinates (0-based node index, x fastest), each of shape [nz, ny, nx]."""
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) == 3 else 1
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def slab_profile(x, nx, rho_L, rho_V, SV, W):
    """eq. eqInit: central liquid slab with vapor saturation SV, width W."""
    return rho_V + 0.5 * (rho_L - rho_V) * (np.tanh(2.0 * (x - 0.5 * SV * nx) / W)
                                            - np.tanh(2.0 * (x - (1.0 - 0.5 * SV) * nx) / W))


def droplet_indicator(r, R0, W):
    """eq. eqInit2D written as a 0..1 indicator: 1/2 - 1/2 tanh(2 (r - R0) / W)."""
    return 0.5 - 0.5 * np.tanh(2.0 * (r - R0) / W)


def initial_field(w: Workload, seed=None, rho_LV=None):
    """Molar densities [nc, nz, ny, nx] and velocity [D, nz, ny, nx] (or None)."""
    x, y, z = _grid(w.shape)
    if w.geometry == "uniform":
        # a uniform state with a seeded multiplicative fluctuation of the total
        # density (the composition stays uniform)
        r0 = np.array(states()[w.state_key]["state"]["rho_uniform"])
        rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
        fluct = 1.0 + w.noise * rng.uniform(-1.0, 1.0, x.shape)
        return np.ascontiguousarray(np.stack([r0[i] * fluct for i in range(len(r0))])), None
    rho_L, rho_V, _ = w.phase_densities() if rho_LV is None else (*rho_LV, None)
    nx, ny = w.shape[0], w.shape[1]
    nz = w.shape[2] if len(w.shape) == 3 else 1
    nc = len(rho_L)
    u = None
    if w.geometry == "slab":
        rho = np.stack([slab_profile(x, nx, rho_L[i], rho_V[i], w.vapor_saturation, w.W) for i in range(nc)])
    elif w.geometry == "droplet":
        xc, yc, zc = nx / 2.0, ny / 2.0, nz / 2.0
        r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2 / w.h ** 2 + ((z - zc) ** 2 if nz > 1 else 0.0))
        phi = droplet_indicator(r, w.radius, w.W)
        rho = np.stack([rho_V[i] + (rho_L[i] - rho_V[i]) * phi for i in range(nc)])
    elif w.geometry == "two_droplets":
        xc, yc, zc = nx / 2.0, ny / 2.0, nz / 2.0
        d = 0.5 * w.separation
        rl = np.sqrt((x - (xc - d)) ** 2 + (y - yc) ** 2 + (z - zc) ** 2)
        rr = np.sqrt((x - (xc + d)) ** 2 + (y - yc) ** 2 + (z - zc) ** 2)
        pl = droplet_indicator(rl, w.radius, w.W)
        pr = droplet_indicator(rr, w.radius, w.W)
        phi = np.maximum(pl, pr)
        rho = np.stack([rho_V[i] + (rho_L[i] - rho_V[i]) * phi for i in range(nc)])
        u = np.zeros((3,) + rho.shape[1:])
        u[0] = w.u0 * (pl - pr)          # droplets move toward each other
    else:
        raise ValueError(w.geometry)
    if w.noise:
        rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
        rho = rho * (1.0 + w.noise * rng.uniform(-1.0, 1.0, rho.shape))
    return np.ascontiguousarray(rho), (None if u is None else np.ascontiguousarray(u))


def serving_requests(n=512, seed=0, L_min=64, L_max=2048, ny=8):
    """Seeded request stream for the batched VLE server.

    Each request: lattice L x ny with L log-uniform in [L_min, L_max] (rounded to
    a multiple of 8), feed z1 drawn uniform in [0.05, 0.95] and redrawn while it
    has no S_V = 0.5 two-phase state on the isotherm, and the slab's phase
    densities interpolated from the stored isotherm table.  Returns a list of
    dicts and the number of rejected draws.
    """
    st = states()["binary_isotherm"]
    table = st["table"]
    z1s = np.array([r["z1_at_SV_half"] for r in table])
    order = np.argsort(z1s)
    z1s = z1s[order]
    rows = [table[k] for k in order]
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    rejected = 0
    while len(out) < n:
        L = int(round(math.exp(rng.uniform(math.log(L_min), math.log(L_max))) / 8.0)) * 8
        z1 = rng.uniform(0.05, 0.95)
        if not (z1s[0] <= z1 <= z1s[-1]):
            rejected += 1
            continue
        k = int(np.searchsorted(z1s, z1))
        k = min(max(k, 1), len(rows) - 1)
        t = (z1 - z1s[k - 1]) / (z1s[k] - z1s[k - 1])
        lerp = lambda a, b: (1 - t) * np.asarray(a) + t * np.asarray(b)
        rL = lerp(rows[k - 1]["rho_L"], rows[k]["rho_L"])
        rV = lerp(rows[k - 1]["rho_V"], rows[k]["rho_V"])
        p = float(lerp(rows[k - 1]["p"], rows[k]["p"]))
        out.append({"L": max(L, L_min), "ny": ny, "z1": float(z1), "p": p,
                    "rho_L": rL, "rho_V": rV})
    return out, rejected
