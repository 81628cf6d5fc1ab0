"""CPU replay of the fused step's schedule (the index arithmetic of
k_fused_step, written out here independently): every dependency a block waits
for exists, is produced only by lower-numbered blocks of the same XCD, covers
the stencil's rows and planes, and every node is collided exactly once."""
import itertools

import pytest


def schedule(nx, ny, nz):
    rows_max = (ny + 7) // 8 + 4
    tpp = (rows_max * nx + 255) // 256
    nblocks = (nz + 5) * tpp
    for k in range(8):
        Y0, Y1 = k * ny // 8, (k + 1) * ny // 8
        rowsA = Y1 - Y0 + 4
        produced = {}                      # A-plane index -> set of (z, y) rows
        last_block_of_plane = {}
        collided = []
        for j in range(nblocks):
            a, t = divmod(j, tpp)
            if a < nz + 4:
                z = (a - 2) % nz
                for pos in range(t * 256, min((t + 1) * 256, rowsA * nx)):
                    rl = pos // nx
                    produced.setdefault(a, set()).add((z, (Y0 - 2 + rl) % ny))
                last_block_of_plane[a] = j
            zb = a - 5
            if 0 <= zb < nz:
                need = [zb + q for q in range(5)]
                for q in need:
                    assert q in last_block_of_plane, (k, j, q)          # the counter is incremented
                    assert last_block_of_plane[q] < j or (q == a and False)
                have = set().union(*(produced[q] for q in need))
                for pos in range(t * 256, min((t + 1) * 256, (Y1 - Y0) * nx)):
                    rl, x = divmod(pos, nx)
                    y = Y0 + rl
                    collided.append((x, y, zb))
                    for dz, dy in itertools.product(range(-2, 3), range(-2, 3)):
                        if abs(dz) + abs(dy) <= 2:
                            assert ((zb + dz) % nz, (y + dy) % ny) in have, (k, j, zb, y, dz, dy)
        yield k, collided


@pytest.mark.parametrize("shape", [(32, 64, 16), (48, 72, 9), (16, 67, 12), (32, 64, 20), (16, 96, 5),
                                   (128, 128, 8), (16, 64, 4)])
def test_fused_schedule(shape):
    nx, ny, nz = shape
    seen = []
    for k, c in schedule(nx, ny, nz):
        seen.extend(c)
    assert len(seen) == nx * ny * nz
    assert len(set(seen)) == nx * ny * nz
