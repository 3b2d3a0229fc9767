"""CPU model of how the step kernel finds the reference densities of FP16
storage with a per-node reference (LBM_F16R), checked against the neighbour
table on random images.

The kernel reads one 8-byte window of the reference array per row of the
node's 3x3 row neighbourhood, starting at the even node (r0 - 1) & ~1, where
r0 is the number of fluid voxels before voxel x of that row in node order
(the node of voxel x when it is fluid); each direction takes its source's
entry from its row's window, or the node's own at a wall.  Across the
periodic x wrap (x = 0 or nx - 1, rows of 3 or more voxels) the source is
found instead from the population's gather offset, which the kernel forms
modulo 2^32 from a base `slack` elements below the chunk: the inversion must
hold for states beyond 4 GiB, emulated here with large chunk numbers."""
import numpy as np
import pytest

import paper_1902_11193_amd as P
from lbm_inputs import random_mask


@pytest.mark.parametrize("shape,solid,seed", [((5, 6, 7), 0.3, 1), ((4, 3, 40), 0.5, 2), ((3, 4, 3), 0.2, 3),
                                              ((2, 2, 2), 0.3, 4), ((6, 5, 19), 0.6, 5)])
def test_reference_windows_hold_every_source(shape, solid, seed):
    mask = random_mask(shape, solid, seed)
    nz, ny, nx = mask.shape
    order = P.lbm_node_order(mask)
    nf = len(order)
    if nf == 0:
        return
    node_of = -np.ones(mask.size, np.int64)
    node_of[order] = np.arange(nf)
    node_of = node_of.reshape(mask.shape)
    # r0 of voxel (z, y, x): fluid voxels before it in node order = the node of
    # the first fluid voxel at or after x in its row, or the row's end
    r0 = np.empty(mask.shape, np.int64)
    for z in range(nz):
        for y in range(ny):
            fl = np.flatnonzero(mask[z, y] == 0)
            start = node_of[z, y, fl[0]] if len(fl) else None
            for x in range(nx):
                before = int(np.count_nonzero(mask[z, y, :x] == 0))
                if start is None:   # an empty row: any in-range number; no source comes from it
                    r0[z, y, x] = 0
                else:
                    r0[z, y, x] = start + before
    table = P.lbm_neighbor_table(mask)                       # (18, nf), -1 at a wall
    c = P.lbm_velocities()
    bad = 0
    for n in range(nf):
        v = int(order[n])
        x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
        for i in range(1, 19):
            m = int(table[i - 1, n])
            if m < 0:
                continue                                     # wall: the node's own reference
            dy, dz = -c[i][1], -c[i][2]
            rr0 = int(r0[(z + dz) % nz, (y + dy) % ny, x])
            e = (rr0 - 1 if rr0 > 0 else 0) & ~1
            wrap = nx >= 3 and ((x == 0 and c[i][0] == 1) or (x == nx - 1 and c[i][0] == -1))
            if wrap:
                continue                                     # checked below
            if not e <= m <= e + 3:
                bad += 1
        rr0 = int(r0[z, y, x])
        assert rr0 == n
        e = (rr0 - 1 if rr0 > 0 else 0) & ~1
        assert e <= n <= e + 3
    assert bad == 0


def test_wrapped_source_from_gather_offset_beyond_4gib():
    """node_elem(m) + i * 256 = chunk * 19 * 256 - slack + off / sizeof(T),
    with off formed modulo 2^32 (FP16: 2-byte elements)."""
    rng = np.random.default_rng(7)
    S, K, sz = 19, 256, 2
    checked = 0
    for _ in range(20000):
        npad = int(rng.choice([2560, 144228864, 1 << 30]))
        slack = int(rng.integers(0, 10**8))
        ch = int(rng.integers(0, npad // K))
        m = int(rng.integers(0, npad))
        i = int(rng.integers(1, 19))
        ne_true = (m // K) * S * K + m % K + i * K
        if not 0 <= ne_true - (ch * S * K - slack) < 2**31:
            continue                                     # outside any chunk's gather window
        kb = ((slack - ch * S * K) * sz) % 2**32
        off = (ne_true * sz + kb) % 2**32
        ne = ch * S * K - slack + off // sz - i * K
        assert (ne // (S * K)) * K + ne % (S * K) == m
        checked += 1
    assert checked > 1000
