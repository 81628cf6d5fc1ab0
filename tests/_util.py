"""Shared test helpers: build matching oracle and GPU solvers from a workload."""
import numpy as np

from oracle import lbm
from oracle import lattice as olat
from oracle import thermo as th
from paper_2212_10680_amd import workloads as wl


def mixture_of(w, eos="PR"):
    comps, kij, T = w.thermo()
    return th.Mixture([c["Tc"] for c in comps], [c["Pc"] for c in comps],
                      [c["omega"] for c in comps], T, kij=kij, M=[c["M"] for c in comps],
                      kappa=[c["kappa"] for c in comps], eos=eos)


def oracle_for(w, eos="PR", force_level=0, mrt_S=None):
    return lbm.OracleLBM(mixture_of(w, eos), w.lattice, w.shape, tau=w.tau, collision=w.collision,
                         force_level=force_level, mrt_S=mrt_S)


def direction_map(lattice, gpu_e):
    """perm such that oracle direction perm[a] has the velocity of GPU direction a."""
    oe, _ = olat.lattice(lattice)
    oe3 = np.zeros((oe.shape[0], 3), dtype=int)
    oe3[:, :oe.shape[1]] = oe
    perm = []
    for a in range(gpu_e.shape[0]):
        hit = np.where((oe3 == gpu_e[a]).all(axis=1))[0]
        assert hit.size == 1
        perm.append(int(hit[0]))
    return np.array(perm)


def smooth_3d_field(w, amp=0.01):
    """Workload field times a smooth modulation in y and z (a genuinely 3-D field
    without white noise, which excites the D3Q19 high-wavenumber modes)."""
    rho, u = wl.initial_field(w)
    nx, ny, nz = w.shape
    z, y = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
    mod = 1.0 + amp * np.sin(2 * np.pi * y / ny) * np.cos(2 * np.pi * z / nz)
    return np.ascontiguousarray(rho * mod[None, :, :, None]), u


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
