"""Python driver of the FP64 C oracle (``oracle/lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by tests/, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``.

``OracleLBM`` holds the populations g[c][a][node] and the previous step's total
force, and advances them with the literal nine-step procedure of Sec. III.B.
EOS constants come from :mod:`oracle.thermo` (App. C), lattice tables and the
MRT basis from :mod:`oracle.lattice`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import lattice as lat
from .thermo import Mixture

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

MAXC = 8
MAXQ = 19
EOS_ID = {"PR": 0, "SRK": 1, "VDW": 2}


def build(force=True):
    """Compile the oracle with gcc (-O2, OpenMP, IEEE arithmetic)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [
        ("D", C.c_int), ("Q", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("nc", C.c_int), ("eos", C.c_int), ("collision", C.c_int),
        ("force_level", C.c_int), ("standard_force", C.c_int),
        ("RT", C.c_double), ("tau", C.c_double), ("cs2", C.c_double),
        ("b", C.c_double * MAXC), ("M", C.c_double * MAXC), ("kappa", C.c_double * MAXC),
        ("aaij", C.c_double * (MAXC * MAXC)),
        ("e", C.c_double * (MAXQ * 3)), ("w", C.c_double * MAXQ),
        ("Mm", C.c_double * (MAXQ * MAXQ)), ("Minv", C.c_double * (MAXQ * MAXQ)),
        ("S", C.c_double * MAXQ),
        ("stencil", C.c_int),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        _lib = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        _lib.orc_run.argtypes = [C.POINTER(_Params), dp, dp, C.c_long,
                                 C.POINTER(C.c_long), C.POINTER(C.c_long)]
        _lib.orc_run.restype = C.c_int
        _lib.orc_init.argtypes = [C.POINTER(_Params), dp, dp, dp, dp]
        _lib.orc_init.restype = None
        _lib.orc_fields.argtypes = [C.POINTER(_Params), dp, dp, dp, dp, dp, dp, dp, dp]
        _lib.orc_fields.restype = C.c_int
        _lib.orc_eos.argtypes = [C.POINTER(_Params), dp, dp, dp]
        _lib.orc_eos.restype = C.c_int
        _lib.orc_equilibrium.argtypes = [C.POINTER(_Params), C.c_double, dp, dp]
        _lib.orc_equilibrium.restype = None
        _lib.orc_forcing.argtypes = [C.POINTER(_Params), dp, dp, dp, dp]
        _lib.orc_forcing.restype = None
        _lib.orc_num_threads.argtypes = []
        _lib.orc_num_threads.restype = C.c_int
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_set_threads.restype = None
        _lib.orc_iso_stencils.argtypes = [C.POINTER(_Params), dp, dp, dp]
        _lib.orc_iso_stencils.restype = None
    return _lib


def num_threads():
    return _load().orc_num_threads()


def set_threads(n):
    """Host threads the oracle's OpenMP loops use from now on."""
    _load().orc_set_threads(int(n))


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleLBM:
    """FP64 oracle lattice.

    mixture   : :class:`oracle.thermo.Mixture` (with M and kappa set)
    lattice   : 'D2Q9' or 'D3Q19'
    shape     : (nx, ny) or (nx, ny, nz)
    collision : 'BGK' or 'MRT' (rates from :func:`oracle.lattice.mrt_rates`
                unless ``mrt_S`` is given)
    force_level : 0 = previous step's force in u (literal step 1), 1 = same step
    standard_force : use the standard-LBM force variant (eqForceGen)
    stencil   : 'axis' (the paper's eq1stder / eq2ndder) or 'isotropic'
                (lattice-weighted stencils; a reading for 3-D droplets, which
                leave the EOS domain with the axis stencils)
    """

    def __init__(self, mixture: Mixture, lattice="D2Q9", shape=(64, 8), tau=1.0,
                 collision="BGK", force_level=0, mrt_S=None, standard_force=False, stencil="axis"):
        self.mix = mixture
        self.lattice = lattice
        e, w = lat.lattice(lattice)
        self.D = e.shape[1]
        self.Q = e.shape[0]
        shape = tuple(int(s) for s in shape)
        if len(shape) == 2:
            shape = shape + (1,)
        assert len(shape) == 3 and (self.D == 3 or shape[2] == 1)
        self.shape = shape
        self.N = shape[0] * shape[1] * shape[2]
        nc = mixture.n
        self.nc = nc
        assert nc <= MAXC
        P = _Params()
        P.D, P.Q = self.D, self.Q
        P.nx, P.ny, P.nz = shape
        P.nc = nc
        P.eos = EOS_ID[mixture.eos]
        P.collision = 1 if collision == "MRT" else 0
        P.force_level = int(force_level)
        P.standard_force = int(bool(standard_force))
        if stencil not in ("axis", "isotropic"):
            raise ValueError(stencil)
        P.stencil = 1 if stencil == "isotropic" else 0
        P.RT = mixture.RT
        P.tau = float(tau)
        P.cs2 = lat.CS2
        kappa = mixture.kappa if mixture.kappa is not None else np.zeros(nc)
        for i in range(nc):
            P.b[i] = mixture.b[i]
            P.M[i] = mixture.M[i]
            P.kappa[i] = kappa[i]
            for j in range(nc):
                P.aaij[i * nc + j] = mixture.aaij[i, j]
        for a in range(self.Q):
            for k in range(3):
                P.e[3 * a + k] = float(e[a, k]) if k < self.D else 0.0
            P.w[a] = w[a]
        if collision == "MRT":
            Mm, _ = lat.mrt_basis(lattice)
            Minv = np.linalg.inv(Mm)
            S = lat.mrt_rates(lattice, tau) if mrt_S is None else np.asarray(mrt_S, float)
            for k in range(self.Q):
                P.S[k] = S[k]
                for a in range(self.Q):
                    P.Mm[k * self.Q + a] = Mm[k, a]
                    P.Minv[k * self.Q + a] = Minv[k, a]
        self.params = P
        self.g = np.zeros((nc, self.Q, self.N))
        self.fprev = np.zeros((self.D, self.N))
        self.steps = 0

    # ------------------------------------------------------------- state
    def init(self, rho_molar, u=None):
        """g = g_eq(rho_i, u), zero force history (the paper does not say how the
        populations are initialised; equilibrium is the reading used)."""
        rho = np.ascontiguousarray(np.asarray(rho_molar, dtype=np.float64).reshape(self.nc, self.N))
        uu = None
        if u is not None:
            uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(self.D, self.N))
        _load().orc_init(C.byref(self.params), _ptr(rho), _ptr(uu), _ptr(self.g), _ptr(self.fprev))
        self.steps = 0

    def run(self, nsteps):
        done = C.c_long(0)
        bad = C.c_long(-1)
        err = _load().orc_run(C.byref(self.params), _ptr(self.g), _ptr(self.fprev),
                              int(nsteps), C.byref(done), C.byref(bad))
        self.steps += done.value
        if err != 0:
            raise FloatingPointError(f"oracle domain error {err} at node {bad.value} "
                                     f"after {done.value} steps")
        return self

    def fields(self):
        """dict of rho_molar [nc,N], u [D,N], p [N], lnf [nc,N], force [nc,D,N], mu_I [nc,N]."""
        nc, D, N = self.nc, self.D, self.N
        out = {"rho_molar": np.zeros((nc, N)), "u": np.zeros((D, N)), "p": np.zeros(N),
               "lnf": np.zeros((nc, N)), "force": np.zeros((nc, D, N)), "mu_I": np.zeros((nc, N))}
        err = _load().orc_fields(C.byref(self.params), _ptr(self.g), _ptr(self.fprev),
                                 _ptr(out["rho_molar"]), _ptr(out["u"]), _ptr(out["p"]),
                                 _ptr(out["lnf"]), _ptr(out["force"]), _ptr(out["mu_I"]))
        if err != 0:
            raise FloatingPointError(f"oracle domain error {err}")
        return out

    def mass(self):
        """Total mass of each component, sum over nodes and directions."""
        return self.g.sum(axis=(1, 2))

    def reshape_field(self, f):
        """[..., N] -> [..., nz, ny, nx] (x fastest)."""
        nx, ny, nz = self.shape
        return f.reshape(f.shape[:-1] + (nz, ny, nx))

    def iso_stencils(self, f):
        """The isotropic lattice stencils of the scalar field f [N] on this
        lattice: (grad [D, N], lap [N])."""
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(self.N))
        grad = np.zeros((3, self.N))
        lap = np.zeros(self.N)
        _load().orc_iso_stencils(C.byref(self.params), _ptr(f), _ptr(grad), _ptr(lap))
        return grad[:self.D], lap

    # --------------------------------------------------- single-node pieces
    def eos(self, rho_molar):
        rho = np.ascontiguousarray(np.asarray(rho_molar, dtype=np.float64))
        p = np.zeros(1)
        lnf = np.zeros(self.nc)
        err = _load().orc_eos(C.byref(self.params), _ptr(rho), _ptr(p), _ptr(lnf))
        if err != 0:
            raise FloatingPointError("domain")
        return p[0], lnf

    def equilibrium(self, rho_i, u):
        u3 = np.zeros(3)
        u3[:len(u)] = u
        geq = np.zeros(self.Q)
        _load().orc_equilibrium(C.byref(self.params), float(rho_i), _ptr(u3), _ptr(geq))
        return geq

    def forcing(self, F, grho, u):
        F3, g3, u3 = np.zeros(3), np.zeros(3), np.zeros(3)
        F3[:len(F)] = F
        g3[:len(grho)] = grho
        u3[:len(u)] = u
        Fa = np.zeros(self.Q)
        _load().orc_forcing(C.byref(self.params), _ptr(F3), _ptr(g3), _ptr(u3), _ptr(Fa))
        return Fa
