"""CPU replay of the z-marching collide/stream kernel's data staging.

The kernel (k_collide_zmarch) gives each 256-thread workgroup a 64 x 4 tile of
(x, y) and a range of z planes, marched upward or downward, keeps phi in a
4-slot LDS ring (tile + halo 2), rt and ln f in a 2-slot ring (tile + halo 1),
and the node's own column at z +- 1, z +- 2 in registers (the values ahead
loaded one plane early, with the node's populations).  This replays that
schedule with the kernel's index arithmetic (fill offsets, slot numbers,
register shifts, block order over the XCDs) and checks, for every node of every
plane, that each value the stencil reads is the field at the periodic neighbour
the stencil means, and that every LDS and global index stays inside its buffer.
"""
import numpy as np
import pytest

ZX, ZY = 64, 4
PHI_W, PHI_H = ZX + 4, ZY + 4
RL_W, RL_H = ZX + 2, ZY + 2
PHI_PTS, RL_PTS = PHI_W * PHI_H, RL_W * RL_H
PHI_PER, RL_PER = (PHI_PTS + 255) // 256, (RL_PTS + 255) // 256

PHI_OFFS = [(dx, dy, dz) for dx in range(-2, 3) for dy in range(-2, 3) for dz in range(-2, 3)
            if abs(dx) + abs(dy) + abs(dz) <= 2]
RL_OFFS = [(0, 0, 0)] + [tuple(s * (k == m) for m in range(3)) for k in range(3) for s in (1, -1)]


def wrap2(v, m):
    v = np.where(v < 0, v + m, v)
    v = np.where(v < 0, v + m, v)
    v = np.where(v >= m, v - m, v)
    return np.where(v >= m, v - m, v)


def replay(nx, ny, nz, zlen, remap=True, direction=1):
    rng = np.random.default_rng(nx * 1000 + ny * 10 + nz)
    phi = rng.standard_normal((nz, ny, nx))
    rl = rng.standard_normal((nz, ny, nx))   # one rt / ln f field stands for all
    plane = nx * ny
    tiles_x = nx // ZX
    tiles_xy = tiles_x * (ny // ZY)
    nzc = (nz + zlen - 1) // zlen
    nb = tiles_xy * nzc
    chunk = (nb + 7) // 8 if remap else 0
    grid = 8 * chunk if remap else nb
    seen = []
    flat_phi, flat_rl = phi.reshape(-1), rl.reshape(-1)
    t = np.arange(256)
    tx, ty = t % ZX, t // ZX
    visits = np.zeros((nz, ny, nx), dtype=int)
    D = direction
    for b in range(grid):
        j = b >> 3
        lb = (b & 7) * chunk + (j if D > 0 else chunk - 1 - j) if remap else b
        if lb >= nb:
            continue
        seen.append(lb)
        zc, txy = lb // tiles_xy, lb % tiles_xy
        x0, y0 = (txy % tiles_x) * ZX, (txy // tiles_x) * ZY
        z0, z1 = zc * zlen, min(zc * zlen + zlen, nz)
        start = z0 if D > 0 else z1 - 1
        x, y = x0 + tx, y0 + ty
        col = x + nx * y
        phi_off, rl_off = [], []
        for k in range(PHI_PER):
            p = t + 256 * k
            phi_off.append(np.where(p < PHI_PTS, wrap2(x0 - 2 + p % PHI_W, nx) + nx * wrap2(y0 - 2 + p // PHI_W, ny), -1))
        for k in range(RL_PER):
            p = t + 256 * k
            rl_off.append(np.where(p < RL_PTS, wrap2(x0 - 1 + p % RL_W, nx) + nx * wrap2(y0 - 1 + p // RL_W, ny), -1))
        for o in phi_off + rl_off:
            assert np.all((o == -1) | ((o >= 0) & (o < plane)))

        def zoff(zz):
            z = int(wrap2(np.array(zz), nz))
            assert 0 <= z < nz
            return z * plane

        s_phi = np.full((4, PHI_PTS), np.nan)
        s_rl = np.full((2, RL_PTS), np.nan)

        def fill(dst, slot, src, offs):
            for k, o in enumerate(offs):
                m = o >= 0
                idx = (t + 256 * k)[m]
                assert idx.max() < dst.shape[1]
                dst[slot, idx] = src[o[m]]

        for d in range(3):
            fill(s_phi, d, flat_phi[zoff(start + (d - 1) * D):], phi_off)
        fill(s_rl, 0, flat_rl[zoff(start):], rl_off)
        phi_b2 = flat_phi[zoff(start - 2 * D) + col]
        phi_b1 = flat_phi[zoff(start - D) + col]
        rl_b1 = flat_rl[zoff(start - D) + col]
        # the own column ahead is loaded one plane early (the first before the loop)
        phi_a2 = flat_phi[zoff(start + 2 * D) + col]
        rl_a1 = flat_rl[zoff(start + D) + col]
        cphi = (ty + 2) * PHI_W + tx + 2
        crl = (ty + 1) * RL_W + tx + 1
        for it in range(z1 - z0):
            zz = start + it * D
            fphi = [np.where(o >= 0, flat_phi[zoff(zz + 2 * D) + np.maximum(o, 0)], 0.0) for o in phi_off]
            frl = [np.where(o >= 0, flat_rl[zoff(zz + D) + np.maximum(o, 0)], 0.0) for o in rl_off]
            s0, r0 = (it + 1) & 3, it & 1
            for dx, dy, dz in PHI_OFFS:
                d = dz * D
                if d == -2:
                    got = phi_b2
                elif d == 2:
                    got = phi_a2
                else:
                    i = cphi + dy * PHI_W + dx
                    assert i.min() >= 0 and i.max() < PHI_PTS
                    got = s_phi[(s0 + d) & 3, i]
                want = phi[wrap2(zz + dz, nz), wrap2(y + dy, ny), wrap2(x + dx, nx)]
                np.testing.assert_array_equal(got, want, err_msg=f"phi {dx, dy, dz} z={zz}")
            for dx, dy, dz in RL_OFFS:
                d = dz * D
                if d == -1:
                    got = rl_b1
                elif d == 1:
                    got = rl_a1
                else:
                    i = crl + dy * RL_W + dx
                    assert i.min() >= 0 and i.max() < RL_PTS
                    got = s_rl[r0, i]
                want = rl[wrap2(zz + dz, nz), wrap2(y + dy, ny), wrap2(x + dx, nx)]
                np.testing.assert_array_equal(got, want, err_msg=f"rl {dx, dy, dz} z={zz}")
            n = col + zz * plane
            assert n.min() >= 0 and n.max() < plane * nz
            visits[zz, y, x] += 1
            if it + 1 < z1 - z0:  # the next plane's node inputs and own column
                nn = col + (zz + D) * plane
                assert z0 <= zz + D < z1 and nn.min() >= 0 and nn.max() < plane * nz
                phi_a2 = flat_phi[zoff(zz + 3 * D) + col]
                rl_a1 = flat_rl[zoff(zz + 2 * D) + col]
            phi_b2, phi_b1 = phi_b1, s_phi[s0, cphi]
            rl_b1 = s_rl[r0, crl]
            for k in range(PHI_PER):
                m = phi_off[k] >= 0
                s_phi[(it + 3) & 3, (t + 256 * k)[m]] = fphi[k][m]
            for k in range(RL_PER):
                m = rl_off[k] >= 0
                s_rl[(it + 1) & 1, (t + 256 * k)[m]] = frl[k][m]
    assert sorted(seen) == list(range(nb))
    assert np.all(visits == 1)


@pytest.mark.parametrize("nx,ny,nz,zlen", [
    (64, 4, 1, 16),     # one plane: every z neighbour is the plane itself
    (64, 4, 2, 16),
    (64, 8, 5, 2),      # ragged last z-range
    (128, 8, 9, 4),
    (64, 12, 16, 16),   # three tile rows, one z-range
    (128, 4, 7, 3),
    (192, 8, 6, 5),
])
@pytest.mark.parametrize("direction", [1, -1])
def test_zmarch_schedule(nx, ny, nz, zlen, direction):
    replay(nx, ny, nz, zlen, direction=direction)


@pytest.mark.parametrize("direction", [1, -1])
def test_zmarch_schedule_no_remap(direction):
    replay(64, 8, 6, 4, remap=False, direction=direction)
