"""Pins of the thermodynamics oracle against what the paper and the mathematics fix.

Each test would fail for a plausible slip in ``oracle/thermo.py`` (a dropped
term, a sign, an index, a wrong root): closed forms, identities that hold for
any correct EOS/fugacity pair, an independent quadrature route, a brute-force
Maxwell construction, and the density ratio the paper prints.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import thermo as th

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_pins.json")))


def _binary(eos="PR", kij=0.0):
    Tc, Pc = th.critical_from_ab([2 / 49, 4 / 49], [2 / 21, 2 / 21], eos)
    k = np.array([[0.0, kij], [kij, 0.0]])
    return th.Mixture(Tc, Pc, [0.011, 0.152], 0.8 * Tc[1], kij=k, eos=eos)


def _ternary(eos="PR"):
    Tc, Pc = th.critical_from_ab([2 / 49, 3 / 49, 4 / 49], [2 / 21] * 3, eos)
    k = np.full((3, 3), 0.02) - 0.02 * np.eye(3)
    return th.Mixture(Tc, Pc, [0.011, 0.10, 0.20], 0.85 * Tc[2], kij=k, eos=eos)


STATES = [np.array([1.2, 3.1]), np.array([0.4, 0.25]), np.array([1e-3, 2e-3]),
          np.array([2.5, 4.0])]


@pytest.mark.parametrize("eos,Zc", [("PR", 0.307401), ("SRK", 1.0 / 3.0), ("VDW", 3.0 / 8.0)])
def test_critical_point(eos, Zc):
    """At T = Tc the isotherm has an inflection with zero slope at p = Pc (App. C.1)."""
    Tc, Pc = 300.0, 40.0
    m = th.Mixture([Tc], [Pc], [0.2], Tc, eos=eos, R=th.R_CM3_BAR)
    x = np.array([1.0])
    v = Zc * th.R_CM3_BAR * Tc / Pc
    h = 1e-4 * v
    p0 = m.pressure_v(v, x)
    d1 = (m.pressure_v(v + h, x) - m.pressure_v(v - h, x)) / (2 * h)
    d2 = (m.pressure_v(v + h, x) - 2 * p0 + m.pressure_v(v - h, x)) / h**2
    assert abs(p0 / Pc - 1.0) < 2e-6
    assert abs(d1 * v / Pc) < 2e-5
    assert abs(d2 * v * v / Pc) < 2e-4
    if eos == "PR":
        assert Zc == GOLD["pr_critical_compressibility"]["value"]


@pytest.mark.parametrize("eos", ["PR", "SRK", "VDW"])
@pytest.mark.parametrize("k", range(len(STATES)))
def test_density_form_equals_z_form(eos, k):
    """Sec. V density-explicit ln f == ln x + ln p + App. C.2 Z-form ln phi when p > 0."""
    m = _binary(eos)
    rho = STATES[k]
    p = m.pressure(rho)
    if p <= 0:
        pytest.skip("Z-form needs p > 0")
    x = rho / rho.sum()
    lhs = m.lnf(rho)
    rhs = np.log(x) + math.log(p) + m.lnphi_vp(1.0 / rho.sum(), p, x)
    assert np.max(np.abs(lhs - rhs)) < 1e-12


@pytest.mark.parametrize("eos", ["PR", "SRK", "VDW"])
def test_lnphi_by_quadrature(eos):
    """eq. eqfug2 integrated numerically from the EOS pressure alone."""
    for m, rho in ((_binary(eos), np.array([1.2, 3.1])), (_binary(eos), np.array([0.3, 0.2])),
                   (_ternary(eos), np.array([0.4, 1.1, 2.6]))):
        p = m.pressure(rho)
        if p <= 0:
            continue
        x = rho / rho.sum()
        direct = m.lnf(rho) - np.log(x) - math.log(p)
        quad = m.lnphi_quadrature(rho)
        assert np.max(np.abs(direct - quad)) < 1e-9, (direct, quad)


@pytest.mark.parametrize("mk", [_binary, _ternary])
@pytest.mark.parametrize("eos", ["PR", "SRK", "VDW"])
def test_gibbs_duhem_and_symmetry(mk, eos):
    """dp = sum_i rho~_i d(RT ln f_i) at constant T (Gibbs-Duhem, eq. eqGibbsDuhem),
    and d ln f_i / d rho~_j is symmetric (mu_i is a gradient of a free energy)."""
    m = mk(eos)
    rng = np.random.default_rng(7)
    for _ in range(5):
        rho = rng.uniform(0.2, 3.0 / m.n, m.n)
        J = np.zeros((m.n, m.n))
        for j in range(m.n):
            h = 1e-6 * rho[j]
            e = np.zeros(m.n)
            e[j] = h
            J[:, j] = (m.lnf(rho + e) - m.lnf(rho - e)) / (2 * h)
            dp = (m.pressure(rho + e) - m.pressure(rho - e)) / (2 * h)
            assert abs(dp - m.RT * rho @ J[:, j]) < 1e-7 * max(1.0, abs(dp))
        assert np.max(np.abs(J - J.T)) < 1e-6 * np.max(np.abs(J))


def test_ideal_gas_limit():
    """eq. eqfugdef2: f_i -> x_i p -> rho~_i RT as the density vanishes."""
    m = _ternary()
    for scale in (1e-6, 1e-8):
        rho = scale * np.array([0.2, 0.3, 0.5])
        dev = m.lnf(rho) - np.log(rho * m.RT)
        assert np.max(np.abs(dev)) < 50 * scale


def test_maxwell_vs_fugacity_pure():
    """Pure component: equal-area construction (EOS only) == equal fugacities."""
    Tc, Pc = th.critical_from_ab([4 / 49], [2 / 21])
    m = th.Mixture(Tc, Pc, [0.152], 0.8 * Tc[0])
    pm, vLm, vVm = th.maxwell_equal_area(m)
    pf, vLf, vVf = th.saturation_by_fugacity(m)
    assert abs(pm / pf - 1) < 1e-10
    assert abs(vLm / vLf - 1) < 1e-9 and abs(vVm / vVf - 1) < 1e-9


def test_paper_density_ratio():
    """Sec. IV.E: PR flash of C3/nC5 at 340 K and 5 bar has density ratio 50.97."""
    pin = GOLD["oscillating_droplet_density_ratio"]
    tab = GOLD["table_tabCompProp"]
    c3, c5 = tab["C3"], tab["nC5"]
    m = th.Mixture([c3[1], c5[1]], [c3[0], c5[0]], [c3[2], c5[2]], pin["T_K"], R=th.R_CM3_BAR,
                   M=[c3[3], c5[3]])
    fr = th.flash(m, [0.5, 0.5], pin["p_bar"])
    assert fr.two_phase
    ratio = (fr.rhoL * (fr.x @ m.M)) / (fr.rhoV * (fr.y @ m.M))
    assert abs(ratio - pin["value"]) < 0.005


@pytest.mark.parametrize("mk,z,p", [(_binary, [0.3, 0.7], 0.1185625620521015),
                                    (_ternary, [0.2, 0.3, 0.5], 0.10570467)])
def test_flash_consistency(mk, z, p):
    """Flash result: equal fugacities, material balance, both phases on the EOS."""
    m = mk()
    fr = th.flash(m, z, p)
    assert fr.two_phase
    lnfL = m.lnf(fr.x / fr.vL)
    lnfV = m.lnf(fr.y / fr.vV)
    assert np.max(np.abs(lnfL - lnfV)) < 1e-10
    assert np.max(np.abs(fr.beta * fr.y + (1 - fr.beta) * fr.x - np.array(z))) < 1e-12
    assert abs(m.pressure(fr.x / fr.vL) / p - 1) < 1e-10
    assert abs(m.pressure(fr.y / fr.vV) / p - 1) < 1e-10


def test_rachford_rice_binary_closed_form():
    """Binary Rachford-Rice has the closed form beta = (z1 (K1-K2)/(1-K2) - 1)... (lever rule)."""
    z = np.array([0.3, 0.7])
    K = np.array([2.9, 0.48])
    beta = th.rachford_rice(z, K)
    x1 = (1 - K[1]) / (K[0] - K[1])
    y1 = K[0] * x1
    assert abs(beta - (z[0] - x1) / (y1 - x1)) < 1e-14
