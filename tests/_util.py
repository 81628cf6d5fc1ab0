"""Shared test helpers: build matching oracle and GPU solvers from a workload."""
import numpy as np

from oracle import lbm
from oracle import lattice as olat
from oracle import thermo as th
from paper_2212_10680_amd import workloads as wl


def mixture_of(w, eos=None):
    eos = eos or w.eos
    comps, kij, T = w.thermo()
    return th.Mixture([c["Tc"] for c in comps], [c["Pc"] for c in comps],
                      [c["omega"] for c in comps], T, kij=kij, M=[c["M"] for c in comps],
                      kappa=[c["kappa"] for c in comps], eos=eos)


def oracle_for(w, eos=None, force_level=0, mrt_S=None, standard_force=False, stencil="axis"):
    return lbm.OracleLBM(mixture_of(w, eos), w.lattice, w.shape, tau=w.tau, collision=w.collision,
                         force_level=force_level, mrt_S=mrt_S, standard_force=standard_force,
                         stencil=stencil)


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


def bulk_values(rho):
    """Bulk molar densities of a flat-interface profile (R-17): the mean over
    the central quarter of the liquid and of the vapor region (an even number of
    consecutive nodes), the regions split at rho~ = (max + min) / 2 along the
    periodic axis.  rho: [nc, n] (one row of the lattice).  Returns
    (rho_liquid [nc], rho_vapor [nc])."""
    rho = np.asarray(rho, dtype=np.float64)
    tot = rho.sum(axis=0)
    n = tot.size
    liquid = tot > 0.5 * (tot.max() + tot.min())
    idx = np.arange(n)

    def central(ix):
        # circular mean locates the centre of a region that may wrap around
        c = (np.angle(np.exp(2j * np.pi * ix / n).mean()) * n / (2 * np.pi)) % n
        d = (ix - c + n / 2) % n - n / 2
        sel = ix[np.abs(d) <= 0.125 * ix.size]
        # an even number of consecutive nodes: the even/odd alternation that
        # central differences leave in mu (R-18) cancels in the mean
        if sel.size % 2:
            sel = ix[(np.abs(d) <= 0.125 * ix.size) & (d != d[np.abs(d) <= 0.125 * ix.size].max())]
        return sel

    return rho[:, central(idx[liquid])].mean(axis=1), rho[:, central(idx[~liquid])].mean(axis=1)


def central_pairs(rho):
    """Like bulk_values, but the mean over the two nodes nearest the centre of
    each region only (the narrowest even window).  Returns (rho_liquid [nc],
    rho_vapor [nc])."""
    rho = np.asarray(rho, dtype=np.float64)
    tot = rho.sum(axis=0)
    n = tot.size
    liquid = tot > 0.5 * (tot.max() + tot.min())
    idx = np.arange(n)

    def pair(ix):
        c = (np.angle(np.exp(2j * np.pi * ix / n).mean()) * n / (2 * np.pi)) % n
        d = np.abs((ix - c + n / 2) % n - n / 2)
        return ix[np.argsort(d, kind="stable")[:2]]

    return rho[:, pair(idx[liquid])].mean(axis=1), rho[:, pair(idx[~liquid])].mean(axis=1)


def flash_bulk_pairs(mix, z, rho_L, rho_V, names=("C3", "C5")):
    """Bulk density and mole fractions of each phase with their references
    from a PT flash of the feed z at the liquid bulk's EOS pressure:
    {phase: {"density" | "x_<name>": (value, flash value)}}."""
    fr = th.flash(mix, z, mix.pressure(rho_L))
    assert fr.two_phase
    out = {}
    for phase, r, v, comp in (("liquid", rho_L, fr.vL, fr.x), ("vapor", rho_V, fr.vV, fr.y)):
        d = {"density": (r.sum(), 1.0 / v)}
        for i, n in enumerate(names):
            d["x_" + n] = (r[i] / r.sum(), comp[i])
        out[phase] = d
    return out


def flash_agreement(mix, z, row_a, row_b, names=("C3", "C5")):
    """How the flash errors of two flat-interface states (rows [nc, n]) compare:
    (dq, dref, derr, bound) with dq the largest relative difference of their
    bulk values, dref that of their flash references (each flash is taken at
    its state's own bulk pressure), derr the largest difference of the errors
    (percentage points) and bound its triangle-inequality bound, the largest
    100 (|q - q'| / q_f + q' |q_f - q_f'| / (q_f q_f')).  The errors of the two
    states are equal to within what dq and dref allow when derr <= bound."""
    pa = flash_bulk_pairs(mix, z, *bulk_values(row_a), names)
    pb = flash_bulk_pairs(mix, z, *bulk_values(row_b), names)
    dq = dref = derr = bound = 0.0
    for ph in pa:
        for k, (q, qf) in pa[ph].items():
            qb, qfb = pb[ph][k]
            dq = max(dq, abs(q - qb) / abs(qb))
            dref = max(dref, abs(qf - qfb) / abs(qfb))
            derr = max(derr, abs(100.0 * abs(q - qf) / qf - 100.0 * abs(qb - qfb) / qfb))
            bound = max(bound, 100.0 * (abs(q - qb) / qf + qb * abs(qf - qfb) / (qf * qfb)))
    return dq, dref, derr, bound


def flash_errors_percent(mix, z, rho_L, rho_V, names=("C3", "C5")):
    """Relative errors (eq. eqerror, in %) of bulk density and mole fractions
    against a PT flash of the feed z at the liquid bulk's EOS pressure.
    Keys: "density" and "x_<name>" per component."""
    pairs = flash_bulk_pairs(mix, z, rho_L, rho_V, names)
    return {ph: {k: 100.0 * abs(q - qf) / qf for k, (q, qf) in d.items()} for ph, d in pairs.items()}


def half_width(line, centre, level):
    """Distance from centre to where the profile line (periodic) falls through
    level on each side, by linear interpolation between nodes (the droplet
    boundary of Sec. IV.E); returns the mean of the two sides."""
    n = line.size
    out = []
    for step in (1, -1):
        k = 0
        while line[(centre + step * (k + 1)) % n] >= level:
            k += 1
            if k >= n // 2:
                raise ValueError("no crossing")
        a, b = line[(centre + step * k) % n], line[(centre + step * (k + 1)) % n]
        out.append(k + (a - level) / (a - b))
    return 0.5 * (out[0] + out[1])


def damped_period(t, r, guess):
    """Period of r(t) = c + A exp(-t/d) cos(2 pi t / T + phi) by least squares."""
    from scipy.optimize import curve_fit
    f = lambda t, c, A, d, T, ph: c + A * np.exp(-t / d) * np.cos(2 * np.pi * t / T + ph)
    p0 = [float(np.mean(r)), float(r[0] - np.mean(r)), 4.0 * guess, guess, 0.0]
    p, _ = curve_fit(f, t, r, p0=p0, maxfev=20000)
    return abs(p[3]), p



def swing_statistics(rows, mix, z, names):
    """Per error of eq. eqerror, over sampled rows of a state whose bulk values
    move (the swinging slab of Sec. IV.C, R-26): (mean, std, min, max, window
    shift).  The window shift is the mean difference between the errors from
    the central-quarter bulk window (R-17) and from the two nodes nearest each
    region's centre: the paper does not say where it takes its bulk values."""
    samples = {}
    for r in rows:
        r = np.asarray(r)
        e = flash_errors_percent(mix, z, *bulk_values(r), names=names)
        ep = flash_errors_percent(mix, z, *central_pairs(r), names=names)
        for phase in e:
            for k in e[phase]:
                samples.setdefault((phase, k), []).append((e[phase][k], ep[phase][k]))
    out = {}
    for key, v in samples.items():
        v = np.array(v)
        out[key] = (v[:, 0].mean(), v[:, 0].std(), v[:, 0].min(), v[:, 0].max(), abs((v[:, 1] - v[:, 0]).mean()))
    return out
