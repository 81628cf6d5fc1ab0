"""Per-component mass and rate residual (the FP64 reductions of step 1's
densities) through the C ABI, against the FP64 oracle.

fl_mass returns M_i = sum_x rho_i(x) (Sec. III.B step 1 summed over the
lattice); fl_run_until's residual is r = max_i max_x |rho_i(n) - rho_i(n-K)| /
(K max_x rho_i(n)) over its last K steps.  Both are compared with the same
quantities computed from the oracle's populations at the same step counts, and
the GPU's mass also with an FP64 sum of the GPU's own exported populations
(which pins the reduction itself, independent of how far the two trajectories
drift).  Sizes: a ragged 2-D lattice (two reduction blocks), a 3-D lattice, and
lattices of more than 65 536 nodes, where the final pass folds several block
partials per thread (295 and 529 blocks of 256 nodes).
"""
import numpy as np
import pytest

from paper_2212_10680_amd import fuglbm as F
from paper_2212_10680_amd import workloads as wl

from _util import oracle_for, smooth_3d_field

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def pair(wname, shape, precision="fp64", coll=None):
    w = wl.WORKLOADS[wname].scaled(shape)
    if coll:
        w.collision = coll
    if w.D == 3:
        w.geometry = "slab"
        w.u0 = 0.0
        rho, u = smooth_3d_field(w)
    else:
        rho, u = wl.initial_field(w)
    rho = rho.reshape(w.ncomp, -1)
    u = None if u is None else u.reshape(w.D, -1)
    o = oracle_for(w)
    o.init(rho, u)
    s = F.Solver(F.Params.from_workload(w, precision=precision))
    s.set_state(rho, u)
    return w, o, s


def oracle_densities(o):
    """rho_i(x) = sum_a g_ai(x), [nc, N]."""
    return o.g.sum(axis=1)


CASES = [
    ("binary_slab_2d", (61, 7), 300),          # ragged, 427 nodes
    ("ternary_droplets_3d", (20, 12, 9), 9),   # 3-D, three components
    ("binary_slab_2d", (300, 251), 40),        # 75 300 nodes: 295 partials
    ("ternary_droplet_2d", (520, 260), 20),    # 135 200 nodes: 529 partials
]


@pytest.mark.parametrize("wname,shape,steps", CASES)
def test_mass_vs_oracle(wname, shape, steps):
    announce(f"fl_mass {wname} {shape}")
    w, o, s = pair(wname, shape)
    m0_gpu, m0_orc = s.mass(), o.mass()
    o.run(steps)
    s.step(steps)
    m_gpu, m_orc = s.mass(), o.mass()
    own = s.populations().sum(axis=(1, 2))
    e0 = np.max(np.abs(m0_gpu / m0_orc - 1))
    e1 = np.max(np.abs(m_gpu / m_orc - 1))
    eown = np.max(np.abs(m_gpu / own - 1))
    print(f"  mass at 0: {e0:.1e}; after {steps} steps: vs oracle {e1:.1e}, vs own populations {eown:.1e}; "
          f"drift {np.max(np.abs(m_gpu / m0_gpu - 1)):.1e}", flush=True)
    assert e0 < 1e-13 and e1 < 1e-13 and eown < 1e-13
    s.close()


@pytest.mark.parametrize("wname,shape", [("binary_slab_2d", (300, 251)), ("ternary_droplet_2d", (520, 260))])
def test_mass_fp32_form_matches_its_populations(wname, shape):
    """FP32 populations: the FP64 reduction equals an FP64 sum of the GPU's own
    exported populations (rest slot with its reference added back)."""
    announce(f"fl_mass fp32 {wname} {shape}")
    w, o, s = pair(wname, shape, precision="fp32")
    s.step(25)
    m = s.mass()
    own = s.populations().sum(axis=(1, 2))
    o.run(25)
    e = np.max(np.abs(m / own - 1))
    eo = np.max(np.abs(m / o.mass() - 1))
    print(f"  vs own populations {e:.1e}, vs FP64 oracle {eo:.1e}", flush=True)
    assert e < 1e-13 and eo < 1e-6
    s.close()


@pytest.mark.parametrize("wname,shape,K", [("binary_slab_2d", (61, 7), 50),
                                           ("ternary_droplets_3d", (20, 12, 9), 5),
                                           ("binary_slab_2d", (300, 251), 20),
                                           ("ternary_droplet_2d", (520, 260), 10)])
def test_run_until_residual_vs_oracle(wname, shape, K):
    """Two checks of fl_run_until (tol 0: never converged) after some steps:
    each reported residual against the one computed from oracle densities at
    the same step counts.  Densities agree to ~1e-12 of max rho, so the
    residual (a difference over K steps, divided by K max rho) agrees to a few
    1e-12 / K in absolute terms."""
    announce(f"run_until residual {wname} {shape} K={K}")
    w, o, s = pair(wname, shape)
    s.step(K)
    o.run(K)
    for check in range(2):
        r0 = oracle_densities(o)
        conv, done, res = s.run_until(0.0, K, K)
        o.run(K)
        r1 = oracle_densities(o)
        ref = max(float(np.max(np.abs(r1[i] - r0[i])) / (K * np.max(np.abs(r1[i])))) for i in range(w.ncomp))
        print(f"  check {check}: steps {done} residual GPU {res:.6e} oracle {ref:.6e}", flush=True)
        assert not conv and done == K
        assert ref > 0
        assert abs(res - ref) <= 4e-12 / K + 1e-9 * ref, (res, ref)
    s.close()
