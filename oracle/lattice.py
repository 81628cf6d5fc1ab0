"""Lattice descriptors and MRT moment bases for the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/thermo.py``).

* D2Q9 is the lattice of every simulation in the paper (Sec. IV); weights
  4/9, 1/9, 1/36 and c_s^2 = 1/3 enter eqs. ``eqLBEMCb`` and ``eqLBEMCfinal3``.
* D3Q19 is not used by the paper; the same equations are applied with D = 3 and
  the standard D3Q19 velocities and weights 1/3, 1/18, 1/36.
* MRT is not in the paper either (it uses a single relaxation time in
  eq. ``eqLBEMCa``).  The oracle's MRT reading is m = M g,
  m* = m - S (m - m_eq) + (I - S/2) M Fbar, g* = M^-1 m*, with m_eq = M g_eq
  (the well-balanced equilibrium) and Fbar the full forcing vector of
  eq. ``eqLBEMCfinal3``.  M is the orthogonal polynomial basis of Lallemand &
  Luo (D2Q9) and d'Humieres et al. (D3Q19), built here from its polynomials.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0


def d2q9():
    e = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
                  [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return e, w


def d3q19():
    e = [[0, 0, 0],
         [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
         [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
         [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
         [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]]
    e = np.array(e, dtype=np.int64)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    return e, w


def lattice(name):
    return {"D2Q9": d2q9, "D3Q19": d3q19}[name]()


def mrt_basis(name):
    """Rows of the orthogonal moment basis and the group of each row.

    Groups: 'rho' (conserved), 'j' (momentum), 'nu' (traceless stress),
    'e' (energy / trace of stress), 'ghost' (all higher-order moments).
    """
    e, _ = lattice(name)
    ef = e.astype(np.float64)
    ex, ey = ef[:, 0], ef[:, 1]
    if name == "D2Q9":
        e2 = ex**2 + ey**2
        rows = [
            (np.ones(9), "rho"),
            (-4.0 + 3.0 * e2, "e"),
            (4.0 - 10.5 * e2 + 4.5 * e2**2, "ghost"),   # epsilon
            (ex, "j"),
            ((3.0 * e2 - 5.0) * ex, "ghost"),           # q_x
            (ey, "j"),
            ((3.0 * e2 - 5.0) * ey, "ghost"),           # q_y
            (ex**2 - ey**2, "nu"),
            (ex * ey, "nu"),
        ]
    else:
        ez = ef[:, 2]
        e2 = ex**2 + ey**2 + ez**2
        rows = [
            (np.ones(19), "rho"),
            (19.0 * e2 - 30.0, "e"),
            (12.0 - 26.5 * e2 + 10.5 * e2**2, "ghost"),  # epsilon
            (ex, "j"), ((5.0 * e2 - 9.0) * ex, "ghost"),
            (ey, "j"), ((5.0 * e2 - 9.0) * ey, "ghost"),
            (ez, "j"), ((5.0 * e2 - 9.0) * ez, "ghost"),
            (3.0 * ex**2 - e2, "nu"), ((3.0 * e2 - 5.0) * (3.0 * ex**2 - e2), "ghost"),
            (ey**2 - ez**2, "nu"), ((3.0 * e2 - 5.0) * (ey**2 - ez**2), "ghost"),
            (ex * ey, "nu"), (ey * ez, "nu"), (ex * ez, "nu"),
            ((ey**2 - ez**2) * ex, "ghost"), ((ez**2 - ex**2) * ey, "ghost"),
            ((ex**2 - ey**2) * ez, "ghost"),
        ]
    M = np.array([r for r, _ in rows])
    groups = [g for _, g in rows]
    return M, groups


def mrt_rates(name, tau, s_j=None, s_nu=None, s_e=1.0, s_ghost=1.0):
    """Diagonal of S.  Defaults: s_nu = s_j = 1/tau, s_e = s_ghost = 1."""
    _, groups = mrt_basis(name)
    s_j = 1.0 / tau if s_j is None else s_j
    s_nu = 1.0 / tau if s_nu is None else s_nu
    table = {"rho": 1.0 / tau, "j": s_j, "nu": s_nu, "e": s_e, "ghost": s_ghost}
    return np.array([table[g] for g in groups])
