"""FP64 thermodynamics oracle for the fugacity-based LBM.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
shares no code with it.

Everything here is plain numpy in float64 and follows Appendix C of the paper
(Soomro, Ayala, Peng & Ayala, "A fugacity-based lattice Boltzmann method for
multicomponent multiphase systems", arXiv:2212.10680):

* cubic equations of state (vdW eq. ``eqvdwEOS``, SRK eq. ``eqSRKEOS``,
  PR eq. ``eqPREOS``) with the van der Waals mixing rules
  (eqs. ``eqmixingrulesavdW``, ``eqmixingrulesaSRK``, ``eqmixingrulesbm``);
* the density-explicit log-fugacity the paper recommends for the lattice
  (Sec. V, eqs. ``eqfugupdateVDW``/``eqfugupdateSRK``/``eqfugupdatePR``);
* the Z-form fugacity coefficient (App. C.2, eqs. ``eqfugvdW``/``eqfugSRK``/
  ``eqfugPR``), used by the flash;
* a brute-force route to ln(f_i/(x_i p)) by quadrature of eq. ``eqfug2`` with a
  complex-step derivative of the extensive pressure (no fugacity formula used);
* a PT flash (the paper uses flash calculations but does not give the algorithm:
  Wilson start, successive substitution with Rachford-Rice, Michelsen
  tangent-plane stability), the saturation (S_V) to pressure map used to place a
  slab or droplet, and a brute-force Maxwell equal-area construction for a pure
  component.

Units are whatever the caller uses consistently; the lattice uses R = 1
(Sec. IV: R = 1, a = 2/49, b = 2/21, M = 1 for the most volatile component).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SQRT2 = math.sqrt(2.0)

# Omega_a, Omega_b of each EOS (App. C.1).
OMEGA = {
    "PR": (0.457235529, 0.077796074),
    "SRK": (0.4274802, 0.08664035),
    "VDW": (27.0 / 64.0, 1.0 / 8.0),
}
# Attraction denominator v^2 + u*b*v + w*b^2 of each EOS (App. C.1):
# vdW v^2; SRK v(v+b); PR v^2 + 2bv - b^2.
DENOM_UW = {"PR": (2.0, -1.0), "SRK": (1.0, 0.0), "VDW": (0.0, 0.0)}

# Physical gas constant for the paper's bar / K / cm^3/mol examples.
R_CM3_BAR = 83.14462618

# Critical constants of Table tabCompProp (Pc bar, Tc K, omega, M g/mol).
PAPER_COMPONENTS = {
    "C1": (45.947, 190.74, 0.0104, 16.043),
    "C2": (48.711, 305.51, 0.0979, 30.070),
    "C3": (42.472, 370.03, 0.1522, 44.097),
    "nC5": (33.688, 469.89, 0.2514, 72.150),
}


def alpha_pr(omega, Tr):
    """PR alpha(T) with its two acentric-factor branches (App. C.1, PR)."""
    omega = np.asarray(omega, dtype=np.float64)
    m_lo = 0.374640 + 1.54226 * omega - 0.26992 * omega**2
    m_hi = 0.379642 + 1.48503 * omega - 0.164423 * omega**2 + 0.016666 * omega**3
    m = np.where(omega <= 0.49, m_lo, m_hi)
    return (1.0 + m * (1.0 - np.sqrt(Tr))) ** 2


def alpha_srk(omega, Tr):
    """SRK alpha(T) (App. C.1, SRK)."""
    omega = np.asarray(omega, dtype=np.float64)
    m = 0.48 + 1.574 * omega - 0.176 * omega**2
    return (1.0 + m * (1.0 - np.sqrt(Tr))) ** 2


def critical_from_ab(a, b, eos="PR", R=1.0):
    """Invert a = Oa R^2 Tc^2/Pc, b = Ob R Tc/Pc for (Tc, Pc) (App. C.1)."""
    Oa, Ob = OMEGA[eos]
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    Tc = Ob * a / (Oa * b * R)
    Pc = Ob * R * Tc / b
    return Tc, Pc


@dataclass
class Mixture:
    """A cubic-EOS mixture at fixed temperature T.

    Parameters follow App. C: critical temperature/pressure and acentric factor
    per component, binary interaction coefficients delta_ij (called k_ij in the
    configs; symmetric, zero diagonal), temperature, gas constant R.
    """

    Tc: np.ndarray
    Pc: np.ndarray
    omega: np.ndarray
    T: float
    kij: np.ndarray | None = None
    eos: str = "PR"
    R: float = 1.0
    M: np.ndarray | None = None
    kappa: np.ndarray | None = None
    a: np.ndarray = field(init=False)
    b: np.ndarray = field(init=False)
    alpha: np.ndarray = field(init=False)
    aa: np.ndarray = field(init=False)      # (a alpha)_i
    aaij: np.ndarray = field(init=False)    # (a alpha)_ij

    def __post_init__(self):
        self.Tc = np.atleast_1d(np.asarray(self.Tc, dtype=np.float64))
        self.Pc = np.atleast_1d(np.asarray(self.Pc, dtype=np.float64))
        self.omega = np.atleast_1d(np.asarray(self.omega, dtype=np.float64))
        n = self.Tc.size
        if self.kij is None:
            self.kij = np.zeros((n, n))
        self.kij = np.asarray(self.kij, dtype=np.float64).reshape(n, n)
        if self.M is None:
            self.M = np.ones(n)
        self.M = np.asarray(self.M, dtype=np.float64)
        if self.kappa is not None:
            self.kappa = np.asarray(self.kappa, dtype=np.float64)
        Oa, Ob = OMEGA[self.eos]
        R, T = self.R, self.T
        self.a = Oa * R**2 * self.Tc**2 / self.Pc
        self.b = Ob * R * self.Tc / self.Pc
        Tr = T / self.Tc
        if self.eos == "PR":
            self.alpha = alpha_pr(self.omega, Tr)
        elif self.eos == "SRK":
            self.alpha = alpha_srk(self.omega, Tr)
        else:
            self.alpha = np.ones(n)
        self.aa = self.a * self.alpha
        # (a alpha)_ij = sqrt((a alpha)_i (a alpha)_j) (1 - delta_ij)
        self.aaij = np.sqrt(np.outer(self.aa, self.aa)) * (1.0 - self.kij)

    @property
    def n(self):
        return self.Tc.size

    @property
    def RT(self):
        return self.R * self.T

    # ------------------------------------------------------------------ mixing
    def mix(self, x):
        """(aalpha)_m, b_m and s_i = sum_j x_j (aalpha)_ij (eqs. eqmixingrules*)."""
        x = np.asarray(x, dtype=np.float64)
        s = self.aaij @ x
        am = float(x @ s)
        bm = float(x @ self.b)
        return am, bm, s

    # ---------------------------------------------------------------- pressure
    def pressure_v(self, v, x):
        """p(v, x) from the EOS (eqvdwEOS / eqSRKEOS / eqPREOS)."""
        am, bm, _ = self.mix(x)
        u, w = DENOM_UW[self.eos]
        return self.RT / (v - bm) - am / (v * v + u * bm * v + w * bm * bm)

    def pressure(self, rho):
        """p from the molar densities rho~_i (v = 1/sum rho~_i, x_i = rho~_i/rho~)."""
        rho = np.asarray(rho, dtype=np.float64)
        rt = rho.sum()
        return self.pressure_v(1.0 / rt, rho / rt)

    # ------------------------------------------------- density-explicit ln f
    def lnf(self, rho):
        """ln f_i from the molar densities, density-explicit form of Sec. V.

        PR:  eqfugupdatePR, SRK: eqfugupdateSRK, vdW: eqfugupdateVDW.  These are
        the forms the paper recommends at lattice nodes because the pressure may
        be negative inside interfaces.
        """
        rho = np.asarray(rho, dtype=np.float64)
        rt = rho.sum()
        x = rho / rt
        v = 1.0 / rt
        am, bm, s = self.mix(x)
        RT = self.RT
        b = self.b
        p = self.pressure_v(v, x)
        if self.eos == "VDW":
            return (np.log(x) + b / (v - bm) - np.log((v - bm) / RT)
                    - 2.0 / (RT * v) * s)
        common = np.log(x) + (b / bm) * (p * v / RT - 1.0) - np.log((v - bm) / RT)
        if self.eos == "SRK":
            return common + am / (bm * RT) * (b / bm - 2.0 * s / am) * np.log(1.0 + bm / v)
        return common + am / (2.0 * SQRT2 * bm * RT) * (b / bm - 2.0 * s / am) * np.log(
            (v + (1.0 + SQRT2) * bm) / (v + (1.0 - SQRT2) * bm))

    # ------------------------------------------------------ Z-form ln phi_i
    def lnphi_vp(self, v, p, x):
        """ln(f_i/(x_i p)) at molar volume v, pressure p (eqfugvdW/SRK/PR)."""
        x = np.asarray(x, dtype=np.float64)
        am, bm, s = self.mix(x)
        RT = self.RT
        b = self.b
        if self.eos == "VDW":
            return b / (v - bm) - math.log((v - bm) * p / RT) - 2.0 / (RT * v) * s
        common = (b / bm) * (p * v / RT - 1.0) - math.log((v - bm) * p / RT)
        if self.eos == "SRK":
            return common + am / (bm * RT) * (b / bm - 2.0 * s / am) * math.log(1.0 + bm / v)
        return common + am / (2.0 * SQRT2 * bm * RT) * (b / bm - 2.0 * s / am) * math.log(
            (v + (1.0 + SQRT2) * bm) / (v + (1.0 - SQRT2) * bm))

    # ------------------------------------------------------------ cubic roots
    def volume_roots(self, p, x):
        """All real molar volumes v > b_m with p(v, x) = p, ascending.

        The EOS p = RT/(v-b) - A/D(v) with D = v^2 + u b v + w b^2 is multiplied
        out to p (v-b) D(v) - RT D(v) + A (v-b) = 0 and solved as a cubic.
        """
        am, bm, _ = self.mix(x)
        u, w = DENOM_UW[self.eos]
        D = np.array([1.0, u * bm, w * bm * bm])
        vb = np.array([1.0, -bm])
        poly = p * np.polymul(vb, D)
        poly = np.polysub(poly, self.RT * D)
        poly = np.polyadd(poly, am * vb)
        r = np.roots(poly)
        real = np.sort(r[np.abs(r.imag) <= 1e-9 * np.maximum(1.0, np.abs(r.real))].real)
        real = real[real > bm]
        # polish each root with Newton on the EOS itself
        out = []
        for v in real:
            for _ in range(50):
                f = self.pressure_v(v, x) - p
                h = 1e-7 * v
                df = (self.pressure_v(v + h, x) - self.pressure_v(v - h, x)) / (2 * h)
                if df == 0:
                    break
                dv = f / df
                vn = v - dv
                if vn <= bm:
                    break
                v = vn
                if abs(dv) < 1e-15 * v:
                    break
            out.append(v)
        return np.array(sorted(out))

    def gibbs_root(self, p, x):
        """Root of minimum Gibbs energy sum_i x_i ln f_i among the real roots."""
        roots = self.volume_roots(p, x)
        if roots.size == 1:
            return roots[0]
        x = np.asarray(x, dtype=np.float64)
        g = [float(x @ self.lnphi_vp(v, p, x)) for v in roots]
        return roots[int(np.argmin(g))]

    def lnphi_phase(self, p, x, phase):
        """ln phi_i for a given phase ('L' smallest root, 'V' largest, 'G' min Gibbs)."""
        if phase == "G":
            v = self.gibbs_root(p, x)
        else:
            roots = self.volume_roots(p, x)
            v = roots[0] if phase == "L" else roots[-1]
        return self.lnphi_vp(v, p, x), v

    # --------------------------------------------- quadrature of eqfug2
    def pressure_extensive(self, V, n):
        """p(T, V, n_1..n_N) with x_i = n_i/sum n and v = V/sum n (App. C.2)."""
        ntot = n.sum()
        bm_n = n @ self.b                     # n * b_m
        am_n2 = n @ (self.aaij @ n)           # n^2 * (a alpha)_m
        u, w = DENOM_UW[self.eos]
        return ntot * self.RT / (V - bm_n) - am_n2 / (V * V + u * bm_n * V + w * bm_n * bm_n)

    def lnphi_quadrature(self, rho, npts=400):
        """ln(f_i/(x_i p)) by brute-force quadrature of eq. eqfug2.

        ln phi_i = (1/RT) int_V^inf [(dp/dn_i)_{T,V,n_j} - RT/V] dV - ln Z, with
        (dp/dn_i) from a complex-step derivative of the extensive pressure and
        the integral over V in (V0, inf) mapped to s = V0/V in (0, 1] and done by
        Gauss-Legendre.  Uses only the EOS pressure, no fugacity formula.
        """
        rho = np.asarray(rho, dtype=np.float64)
        n = rho.copy()          # V0 = 1
        V0 = 1.0
        nc = n.size
        xs, ws = np.polynomial.legendre.leggauss(npts)
        s = 0.5 * (xs + 1.0)
        ws = 0.5 * ws
        out = np.zeros(nc)
        h = 1e-30
        for i in range(nc):
            acc = 0.0
            for sk, wk in zip(s, ws):
                V = V0 / sk
                nn = n.astype(np.complex128)
                nn[i] += 1j * h
                dpdn = self.pressure_extensive(V, nn).imag / h
                acc += wk * (dpdn - self.RT / V) * V0 / sk**2
            out[i] = acc / self.RT
        p = self.pressure(rho)
        Z = p * (1.0 / rho.sum()) / self.RT
        return out - math.log(Z)


# ------------------------------------------------------------------ flash
def rachford_rice(z, K):
    """Vapor fraction beta solving sum z_i (K_i-1)/(1+beta(K_i-1)) = 0 (bisection)."""
    z = np.asarray(z, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    lo = 1.0 / (1.0 - K.max())
    hi = 1.0 / (1.0 - K.min())
    f = lambda bt: float(np.sum(z * (K - 1.0) / (1.0 + bt * (K - 1.0))))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 4e-16 * max(1.0, abs(mid)):
            break
    return 0.5 * (lo + hi)


def wilson_k(mix: Mixture, p):
    return mix.Pc / p * np.exp(5.373 * (1.0 + mix.omega) * (1.0 - mix.Tc / mix.T))


def stability_test(mix: Mixture, z, p, tol=1e-12, maxit=2000):
    """Michelsen tangent-plane test.  Returns (unstable, best trial composition)."""
    z = np.asarray(z, dtype=np.float64)
    lnphi_z, _ = mix.lnphi_phase(p, z, "G")
    d = np.log(z) + lnphi_z
    K = wilson_k(mix, p)
    best = (0.0, None)
    for trial in (z * K, z / K):
        Y = trial.copy()
        for _ in range(maxit):
            y = Y / Y.sum()
            lnphi_y, _ = mix.lnphi_phase(p, y, "G")
            Yn = np.exp(d - lnphi_y)
            if np.max(np.abs(np.log(Yn) - np.log(Y))) < tol:
                Y = Yn
                break
            Y = Yn
        y = Y / Y.sum()
        if np.max(np.abs(y - z)) < 1e-6:      # trivial solution
            continue
        if Y.sum() > 1.0 + 1e-9 and Y.sum() - 1.0 > best[0]:
            best = (Y.sum() - 1.0, y)
    return best[1] is not None, best[1]


@dataclass
class FlashResult:
    two_phase: bool
    beta: float            # vapor mole fraction
    x: np.ndarray          # liquid composition
    y: np.ndarray          # vapor composition
    vL: float
    vV: float
    SV: float              # vapor saturation (volume fraction)
    p: float

    @property
    def rhoL(self):
        return 1.0 / self.vL

    @property
    def rhoV(self):
        return 1.0 / self.vV

    @property
    def rho_i_L(self):
        return self.x / self.vL

    @property
    def rho_i_V(self):
        return self.y / self.vV


def flash(mix: Mixture, z, p, tol=1e-13, maxit=100000, check_stability=True):
    """PT flash: stability test, then successive substitution + Rachford-Rice."""
    z = np.asarray(z, dtype=np.float64)
    z = z / z.sum()
    if check_stability:
        unstable, ytrial = stability_test(mix, z, p)
        if not unstable:
            return FlashResult(False, float("nan"), z, z, float("nan"), float("nan"),
                               float("nan"), p)
        K = np.where(ytrial > z, ytrial / z, ytrial / z)
        # the trial phase may be liquid-like or vapor-like; K = y_V/x_L must have
        # both sides of 1; fall back to Wilson if it does not
        if not (K.max() > 1.0 and K.min() < 1.0):
            K = wilson_k(mix, p)
        lnK = np.log(K)
        # orient so that the "vapor" is the less dense phase
        Kw = wilson_k(mix, p)
        if np.dot(np.log(Kw), lnK) < 0:
            lnK = -lnK
    else:
        lnK = np.log(wilson_k(mix, p))
    beta = 0.5
    for it in range(maxit):
        K = np.exp(lnK)
        if not (K.max() > 1.0 and K.min() < 1.0):
            return FlashResult(False, float("nan"), z, z, float("nan"), float("nan"),
                               float("nan"), p)
        beta = rachford_rice(z, K)
        x = z / (1.0 + beta * (K - 1.0))
        y = K * x
        x = x / x.sum()
        y = y / y.sum()
        lphL, vL = mix.lnphi_phase(p, x, "L")
        lphV, vV = mix.lnphi_phase(p, y, "V")
        lnK_new = lphL - lphV
        err = np.max(np.abs(lnK_new - lnK))
        lnK = lnK_new
        if err < tol:
            break
    K = np.exp(lnK)
    beta = rachford_rice(z, K)
    x = z / (1.0 + beta * (K - 1.0))
    y = K * x
    x = x / x.sum()
    y = y / y.sum()
    _, vL = mix.lnphi_phase(p, x, "L")
    _, vV = mix.lnphi_phase(p, y, "V")
    if not (0.0 < beta < 1.0) or abs(vL - vV) < 1e-9 * vL:
        return FlashResult(False, float("nan"), z, z, float("nan"), float("nan"),
                           float("nan"), p)
    SV = beta * vV / (beta * vV + (1.0 - beta) * vL)
    return FlashResult(True, float(beta), x, y, float(vL), float(vV), float(SV), p)


def pressure_for_saturation(mix: Mixture, z, SV_target, p_lo, p_hi, nscan=120,
                            which="lower"):
    """Pressure at which the flash of feed z gives vapor saturation SV_target.

    Scans [p_lo, p_hi] for a sign change of S_V(p) - target (two-phase points
    only) and bisects it; ``which`` picks the lower or upper crossing.
    """
    ps = np.linspace(p_lo, p_hi, nscan)
    vals = []
    for p in ps:
        fr = flash(mix, z, p)
        vals.append(fr.SV - SV_target if fr.two_phase else float("nan"))
    vals = np.array(vals)
    brackets = []
    for k in range(nscan - 1):
        a, b = vals[k], vals[k + 1]
        if np.isfinite(a) and np.isfinite(b) and a * b <= 0.0:
            brackets.append((ps[k], ps[k + 1], a))
    if not brackets:
        raise ValueError("no two-phase state with the requested saturation")
    lo, hi, flo = brackets[0] if which == "lower" else brackets[-1]
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        fr = flash(mix, z, mid)
        fm = fr.SV - SV_target
        if fm * flo > 0.0:
            lo, flo = mid, fm
        else:
            hi = mid
        if hi - lo < 1e-15 * mid:
            break
    p = 0.5 * (lo + hi)
    return p, flash(mix, z, p)


# --------------------------------------------------- pure-component VLE
def maxwell_equal_area(mix: Mixture, npts=2000):
    """Pure-component saturation by brute-force Maxwell equal-area construction.

    Finds p_sat such that int_{vL}^{vV} (p(v) - p_sat) dv = 0, with the loop
    integral done by Gauss-Legendre quadrature of the EOS pressure.  No fugacity
    expression is used.  Returns (p_sat, vL, vV).
    """
    assert mix.n == 1
    x = np.array([1.0])
    b = mix.b[0]
    # spinodal pressures bound p_sat: scan p(v) for its local min/max
    vs = b * np.exp(np.linspace(np.log(1.0001), np.log(1e4), 200000))
    ps = np.array([mix.pressure_v(v, x) for v in vs[::50]])
    vv = vs[::50]
    dp = np.diff(ps)
    imax = np.where((dp[:-1] > 0) & (dp[1:] <= 0))[0]
    imin = np.where((dp[:-1] < 0) & (dp[1:] >= 0))[0]
    p_min = max(ps[imin[0] + 1], 1e-300)
    p_max = ps[imax[0] + 1]
    xs, ws = np.polynomial.legendre.leggauss(npts)

    def area(psat):
        roots = mix.volume_roots(psat, x)
        vL, vV = roots[0], roots[-1]
        # integrate in ln v for accuracy over the wide vapor range
        lo, hi = math.log(vL), math.log(vV)
        t = 0.5 * (hi - lo) * xs + 0.5 * (hi + lo)
        v = np.exp(t)
        integrand = np.array([mix.pressure_v(vi, x) for vi in v]) - psat
        return 0.5 * (hi - lo) * float(np.sum(ws * integrand * v)), vL, vV

    lo, hi = p_min * (1 + 1e-9), p_max * (1 - 1e-9)
    alo = area(lo)[0]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        am, _, _ = area(mid)
        if am * alo > 0:
            lo, alo = mid, am
        else:
            hi = mid
        if hi - lo < 1e-15 * mid:
            break
    psat = 0.5 * (lo + hi)
    _, vL, vV = area(psat)
    return psat, vL, vV


def saturation_by_fugacity(mix: Mixture):
    """Pure-component saturation from ln f_L = ln f_V (bisection on p)."""
    assert mix.n == 1
    x = np.array([1.0])
    psat_m, _, _ = maxwell_equal_area(mix, npts=200)
    lo, hi = psat_m * 0.5, psat_m * 1.5

    def g(p):
        roots = mix.volume_roots(p, x)
        if roots.size < 2:
            return float("nan"), None, None
        vL, vV = roots[0], roots[-1]
        return (mix.lnphi_vp(vL, p, x)[0] - mix.lnphi_vp(vV, p, x)[0]), vL, vV

    # shrink the bracket into the three-root region
    while not np.isfinite(g(lo)[0]):
        lo = 0.5 * (lo + psat_m)
    while not np.isfinite(g(hi)[0]):
        hi = 0.5 * (hi + psat_m)
    glo = g(lo)[0]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        gm = g(mid)[0]
        if gm * glo > 0:
            lo, glo = mid, gm
        else:
            hi = mid
        if hi - lo < 1e-16 * mid:
            break
    p = 0.5 * (lo + hi)
    _, vL, vV = g(p)
    return p, vL, vV


# ----------------------------------------------------- lattice-unit mixtures
def lattice_mixture(a, b, omega, T_over_Tc_of, T_factor, kij=None, M=None, kappa=None,
                    eos="PR"):
    """Mixture specified directly by lattice-unit (a_i, b_i) with R = 1.

    T = T_factor * Tc[T_over_Tc_of] (e.g. 0.8 * Tc of component 2).
    """
    Tc, Pc = critical_from_ab(a, b, eos)
    T = T_factor * Tc[T_over_Tc_of]
    return Mixture(Tc, Pc, omega, T, kij=kij, eos=eos, R=1.0, M=M, kappa=kappa)


def physical_to_lattice(names, eos="PR", a_ref=2.0 / 49.0, b_ref=2.0 / 21.0, R=1.0):
    """Lattice-unit constants of physical components (Sec. IV, conversion rule).

    The paper fixes R = 1 and, for the most volatile component (names[0]),
    a = a_ref, b = b_ref and M = 1.  With a = Oa R^2 Tc^2 / Pc and
    b = Ob R Tc / Pc (App. C) that fixes the lattice Tc and Pc of names[0]; the
    temperature and pressure scales follow, and every other component keeps its
    reduced properties (T/Tc, p/Pc) and its molar-mass ratio.  Component data
    from Table tabCompProp.

    Returns (Tc, Pc, omega, M, T_scale, p_scale): lattice value = physical value
    times the scale (temperatures in K, pressures in bar).
    """
    Tc_ref, Pc_ref = critical_from_ab([a_ref], [b_ref], eos, R)
    Pc_phys = np.array([PAPER_COMPONENTS[n][0] for n in names], dtype=np.float64)
    Tc_phys = np.array([PAPER_COMPONENTS[n][1] for n in names], dtype=np.float64)
    omega = np.array([PAPER_COMPONENTS[n][2] for n in names], dtype=np.float64)
    M_phys = np.array([PAPER_COMPONENTS[n][3] for n in names], dtype=np.float64)
    T_scale = float(Tc_ref[0]) / Tc_phys[0]
    p_scale = float(Pc_ref[0]) / Pc_phys[0]
    return Tc_phys * T_scale, Pc_phys * p_scale, omega, M_phys / M_phys[0], T_scale, p_scale

