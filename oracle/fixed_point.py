"""Discrete equilibrium of the fugacity-based LBM on a 1-D (slab) lattice.

TEST INFRASTRUCTURE ONLY (see ``oracle/thermo.py``).

Derivation (ours, not printed in the paper): with u = 0, every moving
population zero and g_0,i = rho_i, the well-balanced equilibrium (eq. eqLBEMCb
with rho_0 = 0) equals g and the forcing term (eq. eqLBEMCfinal3) reduces to
w_a F_i.e_a / c_s^2.  Such a state is a fixed point of collision and streaming
exactly when F_i = 0 at every node, i.e. (eq. eqforceFugLBM with the central
difference eq1stder) when D(mu_i) = 0 for mu_i = RT ln f_i + mu_I,i and
mu_I,i = -sum_j kappa_ij lap(rho~_j) (eqs. eqChemPotI2, eqkappa, eq2ndder).
On a periodic lattice D(mu) = 0 means mu(x+1) = mu(x-1): mu_i is constant on
the even and on the odd sublattice.  With the odd/even split eta_i and the
component totals N_i given, the state solves

    mu_i(x) = lambda_i + (-1)^x eta_i,      sum_x rho~_i(x) = N_i,

for rho~_i(x) and lambda_i.  This module solves that system by Newton's method
(dense Jacobian; ln f derivatives by central differences of the thermo
oracle's density-explicit ln f, the Laplacian exactly).  It does not depend on
tau, on BGK/MRT or on which time level of the force enters u.
"""
from __future__ import annotations

import numpy as np

from .thermo import Mixture


def _mu(mix: Mixture, rho, kappa):
    """mu_i(x) for rho [nc, n] on a periodic 1-D lattice."""
    nc, n = rho.shape
    kij = np.sqrt(np.outer(kappa, kappa))
    lap = np.roll(rho, -1, axis=1) - 2.0 * rho + np.roll(rho, 1, axis=1)
    lnf = np.stack([mix.lnf(rho[:, x]) for x in range(n)], axis=1)
    return mix.RT * lnf - kij @ lap


def solve(mix: Mixture, rho0, kappa, eta=None, totals=None, tol=1e-14, maxit=60):
    """Newton solve of the discrete equilibrium starting from rho0 [nc, n].

    Returns (rho [nc, n], lambda [nc], final residual max-norm).
    """
    rho = np.array(rho0, dtype=np.float64)
    nc, n = rho.shape
    kappa = np.asarray(kappa, dtype=np.float64)
    eta = np.zeros(nc) if eta is None else np.asarray(eta, dtype=np.float64)
    totals = rho.sum(axis=1) if totals is None else np.asarray(totals, dtype=np.float64)
    sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    mu = _mu(mix, rho, kappa)
    lam = (mu - np.outer(eta, sign)).mean(axis=1)
    kij = np.sqrt(np.outer(kappa, kappa))
    nunk = nc * n + nc
    res_norm = np.inf
    for it in range(maxit):
        mu = _mu(mix, rho, kappa)
        Rm = mu - lam[:, None] - np.outer(eta, sign)
        Rn = rho.sum(axis=1) - totals
        res = np.concatenate([Rm.ravel(), Rn])
        res_norm = np.max(np.abs(res))
        if res_norm < tol:
            break
        J = np.zeros((nunk, nunk))
        # d mu_i(x) / d rho_k(y): local ln f part + Laplacian part
        for x in range(n):
            r = rho[:, x]
            for k in range(nc):
                h = 1e-6 * r[k]
                rp, rm = r.copy(), r.copy()
                rp[k] += h
                rm[k] -= h
                d = mix.RT * (mix.lnf(rp) - mix.lnf(rm)) / (2.0 * h)
                for i in range(nc):
                    J[i * n + x, k * n + x] += d[i]
            for i in range(nc):
                for k in range(nc):
                    J[i * n + x, k * n + x] += 2.0 * kij[i, k]
                    J[i * n + x, k * n + (x + 1) % n] -= kij[i, k]
                    J[i * n + x, k * n + (x - 1) % n] -= kij[i, k]
        for i in range(nc):
            J[i * n:(i + 1) * n, nc * n + i] = -1.0
            J[nc * n + i, i * n:(i + 1) * n] = 1.0
        step = np.linalg.solve(J, -res)
        rho = rho + step[:nc * n].reshape(nc, n)
        lam = lam + step[nc * n:]
    return rho, lam, res_norm


def interfacial_tension(mix: Mixture, rho, kappa, n_interfaces=2):
    """eq. eqMCsigma on a discrete flat-interface profile rho [nc, n] (periodic
    along the row): the integral of sum_ij kappa_ij (d rho~_i/dx)(d rho~_j/dx)
    with central differences (eq1stder) summed over the row, divided by the
    number of interfaces the row holds (a periodic slab has two)."""
    rho = np.asarray(rho, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    kij = np.sqrt(np.outer(kappa, kappa))
    d = 0.5 * (np.roll(rho, -1, axis=1) - np.roll(rho, 1, axis=1))
    return float(np.einsum("ij,ix,jx->", kij, d, d)) / n_interfaces


def lamb_period(sigma, rho_liquid_mass, R_e, n=2):
    """eq. eqPeriod: period of the n-th shape mode of a 2-D droplet,
    T = 2 pi [n (n^2 - 1) sigma / (rho_L R_e^3)]^(-1/2)."""
    return 2.0 * np.pi / np.sqrt(n * (n * n - 1) * sigma / (rho_liquid_mass * R_e ** 3))

