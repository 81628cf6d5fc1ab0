"""CPU replay of the node visiting order of the moments and collide passes.

node_index maps (hardware block, thread) to a logical position: XCD-contiguous
block ranges (hardware block b runs on XCD b mod 8), optionally reversed;
slab_order maps the logical position to a node, y-major inside z-slabs.  The
replay uses the kernels' integer arithmetic and checks that every node of the
lattice is visited exactly once, for shapes whose extents are not multiples of
the block size, the slab depth or 8.
"""
import numpy as np
import pytest


def node_index(b, t, bs, xcd_chunk, N, rev):
    lb = (b & 7) * xcd_chunk + (b >> 3) if xcd_chunk > 0 else b
    if rev:
        lb = (N + bs - 1) // bs - 1 - lb
    n = lb * bs + t
    return np.where((lb < 0) | (n >= N), -1, n)


def slab_order(k, nx, ny, nz, zs):
    if zs <= 0:
        return k
    x = k % nx
    r = k // nx
    per = ny * zs
    sl = r // per
    p = r - sl * per
    zlen = np.minimum(zs, nz - sl * zs)
    y = p // zlen
    z = sl * zs + (p - y * zlen)
    return np.where(k < 0, -1, x + nx * (y + ny * z))


@pytest.mark.parametrize("shape", [(128, 128, 16), (64, 12, 17), (48, 9, 5), (200, 3, 1), (16, 16, 9)])
@pytest.mark.parametrize("bs", [64, 128, 256])
@pytest.mark.parametrize("remap,rev", [(True, False), (True, True), (False, False), (False, True)])
def test_visiting_order_is_a_bijection(shape, bs, remap, rev):
    nx, ny, nz = shape
    N = nx * ny * nz
    nb = (N + bs - 1) // bs
    chunk = (nb + 7) // 8 if remap else 0
    grid = 8 * chunk if remap else nb
    b = np.repeat(np.arange(grid), bs)
    t = np.tile(np.arange(bs), grid)
    zs = (nz + 7) // 8
    n = slab_order(node_index(b, t, bs, chunk, N, rev), nx, ny, nz, zs)
    seen = n[n >= 0]
    assert seen.size == N
    assert np.array_equal(np.sort(seen), np.arange(N))


def test_slab_order_is_y_major_inside_a_slab():
    nx, ny, nz, zs = 4, 3, 5, 2
    k = np.arange(nx * ny * nz)
    n = slab_order(k, nx, ny, nz, zs)
    x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
    rows = list(zip(y[::nx], z[::nx]))
    # slab 0 holds planes 0-1: (y, z) = (0,0),(0,1),(1,0),(1,1),(2,0),(2,1); the
    # last slab (plane 4 alone) comes last
    assert rows[:6] == [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)]
    assert rows[-3:] == [(0, 4), (1, 4), (2, 4)]
    assert np.array_equal(x[:nx], np.arange(nx))


def band_node(b, t, bs, nx, ny, nz, bands, rev):
    """The kernels' XCD-band order: XCD b % 8 sweeps its row bands along z."""
    k, j = b & 7, b >> 3
    maxrows = (ny + bands - 1) // bands
    bpp = (maxrows * nx + bs - 1) // bs
    m = j // (bpp * nz)
    r = j - m * bpp * nz
    z = r // bpp
    q = k + 8 * m
    Y0, Y1 = q * ny // bands, (q + 1) * ny // bands
    pos = (r - z * bpp) * bs + t
    if rev:
        z = nz - 1 - z
    n = pos % nx + nx * (Y0 + pos // nx + ny * z)
    return np.where((m >= bands // 8) | (pos >= (Y1 - Y0) * nx), -1, n)


@pytest.mark.parametrize("shape", [(256, 64, 12), (64, 12, 17), (48, 9, 5), (200, 3, 2), (16, 16, 9), (40, 33, 3)])
@pytest.mark.parametrize("bs", [64, 256])
@pytest.mark.parametrize("bands", [8, 16, 32])
@pytest.mark.parametrize("rev", [False, True])
def test_band_order_is_a_bijection(shape, bs, bands, rev):
    nx, ny, nz = shape
    N = nx * ny * nz
    maxrows = (ny + bands - 1) // bands
    grid = bands * ((maxrows * nx + bs - 1) // bs) * nz
    b = np.repeat(np.arange(grid), bs)
    t = np.tile(np.arange(bs), grid)
    n = band_node(b, t, bs, nx, ny, nz, bands, rev)
    seen = n[n >= 0]
    assert seen.size == N
    assert np.array_equal(np.sort(seen), np.arange(N))


def test_band_order_sweeps_z_inside_a_band():
    """XCD 0's blocks visit band 0's rows plane by plane before its next band."""
    nx, ny, nz, bands, bs = 8, 32, 3, 16, 8
    maxrows = ny // bands
    bpp = maxrows * nx // bs
    b = np.arange(0, 8 * 2 * bpp * nz, 8)          # XCD 0's blocks in dispatch order
    n = np.array([band_node(bb, 0, bs, nx, ny, nz, bands, False) for bb in b])
    y, z = (n // nx) % ny, n // (nx * ny)
    assert list(z[:2 * nz]) == [0, 0, 1, 1, 2, 2]
    assert set(y[:2 * nz]) == {0, 1}
    assert set(y[2 * nz:]) == {16, 17}                # band 8 = XCD 0's second band


def zmarch_tile_of_block(b, tiles_x, tiles_y, nzc, xcd_chunk, zorder):
    """The z-marching kernels' block -> (z-range, tile) map, replayed with their
    integer arithmetic; (-1, -1) for an idle block."""
    if zorder == 1:
        k, j = b & 7, b >> 3
        rows = (tiles_y + 7) >> 3
        per = rows * tiles_x
        zc = j // per
        tl = j - zc * per
        r0, r1 = (k * tiles_y) >> 3, ((k + 1) * tiles_y) >> 3
        ty = r0 + tl // tiles_x
        ok = (zc < nzc) & (ty < r1)
        txy = ty * tiles_x + tl % tiles_x
    else:
        lb = (b & 7) * xcd_chunk + (b >> 3) if xcd_chunk > 0 else b
        zc = lb // (tiles_x * tiles_y)
        txy = lb - zc * tiles_x * tiles_y
        ok = lb < tiles_x * tiles_y * nzc
    return np.where(ok, zc, -1), np.where(ok, txy, -1)


@pytest.mark.parametrize("tiles_x,tiles_y,nzc", [(4, 64, 16), (1, 1, 1), (2, 3, 5), (1, 8, 2), (3, 13, 4),
                                                 (4, 64, 64), (1, 17, 3)])
@pytest.mark.parametrize("zorder", [0, 1])
def test_zmarch_block_order_is_a_bijection(tiles_x, tiles_y, nzc, zorder):
    """Every (z-range, tile) pair of a z-marching launch is taken by exactly
    one block, in the XCD-contiguous and in the XCD y-band order (bands of
    unequal height when the tile rows are not a multiple of 8); in the y-band
    order the blocks of XCD k (b % 8 == k) stay inside band k and take the
    z-ranges in order."""
    nb = tiles_x * tiles_y * nzc
    chunk = (nb + 7) // 8
    grid = 8 * ((tiles_y + 7) // 8) * tiles_x * nzc if zorder == 1 else 8 * chunk
    b = np.arange(grid)
    zc, txy = zmarch_tile_of_block(b, tiles_x, tiles_y, nzc, chunk, zorder)
    ok = zc >= 0
    key = zc[ok] * tiles_x * tiles_y + txy[ok]
    assert key.size == nb
    assert np.array_equal(np.sort(key), np.arange(nb))
    if zorder == 1:
        for k in range(8):
            sel = ok & (b % 8 == k)
            ty = txy[sel] // tiles_x
            assert np.all((ty >= (k * tiles_y) // 8) & (ty < ((k + 1) * tiles_y) // 8))
            assert np.all(np.diff(zc[sel]) >= 0)
