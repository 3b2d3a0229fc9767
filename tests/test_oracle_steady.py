"""Brute-force steady state of the linearised scheme on an 8^3 image, solved
directly and compared with the oracle's time march (Eq. MRT-LBE, Eq. LBE).

With the quadratic terms of the equilibrium and of Guo's source dropped
(the Stokes form, Sec. 2.1.1 after Eq. MRT params) one step is affine in
the gathered populations f:  f' = P (A f + b), where P is the pull stream
with halfway bounce-back and A f + b the collision.  Here P is assembled by
explicit loops over voxels and directions (independent of the oracle's
roll-based stream), A and b by applying the oracle's collision to the 19
unit vectors and to zero (a node-local affine map), and the steady state is
the solution of (I - P A) f = P b.  That system is singular in one
direction, a uniform density change (the rest state is a fixed point of the
unforced map), so it is solved for the deviations d = f - w with
sum(d) = 0 (the march starts at rest and conserves mass) as a bordered sparse
system.  The march reaches it to ~1e-12 of the deviation scale in 1000
steps, averaging two successive steps against the neutral period-2 mode such
images carry; the mass the march has gained by rounding (the numerically
inverted M) is taken out first and checked to be at rounding level.

A mistake in the oracle's stream (a sign of c, the opposite index at a
wall) or in its time loop moves the marched state off the solved one; the
collision itself is pinned by the other oracle tests (moments of the BGK
equilibrium, the MRT-to-BGK reduction, the slit profile)."""
from collections import deque

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl
import torch

import oracle as O
from lbm_inputs import random_mask


def one_component(mask):
    """The largest fluid cluster (18-neighbour links, periodic); all else solid."""
    nz, ny, nx = mask.shape
    fluid = mask == 0
    lab = -np.ones(mask.shape, int)
    links = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
             if 0 < a * a + b * b + c * c <= 2]
    sizes = []
    for start in zip(*np.nonzero(fluid)):
        if lab[start] >= 0:
            continue
        k = len(sizes)
        lab[start] = k
        q, size = deque([start]), 0
        while q:
            z, y, x = q.popleft()
            size += 1
            for cx, cy, cz in links:
                t = ((z + cz) % nz, (y + cy) % ny, (x + cx) % nx)
                if fluid[t] and lab[t] < 0:
                    lab[t] = k
                    q.append(t)
        sizes.append(size)
    out = np.ones_like(mask)
    out[lab == int(np.argmax(sizes))] = 0
    return out


def stream_matrix(mask, c, opp):
    """P acting on [19][N] (entry i*N + k, k = raster order of fluid voxels):
    f_i(x) = fh_i(x - c_i), or fh_opp(i)(x) when x - c_i is solid."""
    nz, ny, nx = mask.shape
    idx = -np.ones(mask.shape, int)
    fl = np.argwhere(mask == 0)
    idx[tuple(fl.T)] = np.arange(len(fl))
    n = len(fl)
    rows, cols = [], []
    for k, (z, y, x) in enumerate(fl):
        for i in range(19):
            cx, cy, cz = c[i]
            s = idx[(z - cz) % nz, (y - cy) % ny, (x - cx) % nx]
            rows.append(i * n + k)
            cols.append(i * n + s if s >= 0 else opp[i] * n + k)
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(19 * n, 19 * n)), n


def collision_affine(p):
    """(A, b) with collide(f) = A f + b at a node (uniform force)."""
    F = p.F[:, :1]
    z = torch.zeros(19, 1, dtype=torch.float64)
    b = O.collide(z, p.s, F, p.lat, linear=True)[:, 0].numpy()
    A = np.empty((19, 19))
    for k in range(19):
        e = z.clone()
        e[k, 0] = 1.0
        A[:, k] = O.collide(e, p.s, F, p.lat, linear=True)[:, 0].numpy() - b
    return A, b


MASK = one_component(random_mask((8, 8, 8), 0.3, 3))
G = (1e-3, 3e-4, -2e-4)


@pytest.mark.parametrize("rset", ["SRT", "A", "B", "C", "D", "E"])
def test_time_march_reaches_direct_steady_solve(rset):
    lat = O.Lattice.make()
    w = lat.w.numpy()
    Pm, n = stream_matrix(MASK, lat.c.numpy(), lat.opp.numpy())
    p = O.Problem(MASK, 0.8, 3 / 16, rset, G, linear=True)
    A, b = collision_affine(p)
    Ab = sp.kron(sp.csr_matrix(A), sp.identity(n), format="csr")
    bb = np.repeat(b, n)
    ones = sp.csr_matrix(np.ones((19 * n, 1)))
    K = sp.bmat([[sp.identity(19 * n) - Pm @ Ab, ones], [ones.T, None]], format="csc")
    sol = spl.spsolve(K, np.concatenate([Pm @ bb, [0.0]]))
    assert abs(sol[-1]) < 1e-15                           # the border multiplier vanishes: consistent system
    f = np.repeat(w, n) + sol[:-1]
    ref = (Ab @ f + bb).reshape(19, n)                    # post-collision steady state
    scale = np.abs(ref - w[:, None]).max()

    fh = p.initial()
    for _ in range(1000):
        prev = fh
        fh, _ = p.step(fh)
    mean = 0.5 * (fh + prev)[:, p.fluid].numpy()
    drift = (mean.sum() - ref.sum()) / n                  # mass gained by rounding, per node
    assert abs(drift) < 1e-12
    err = np.abs(mean - drift * w[:, None] - ref).max() / scale
    assert err < 1e-10, (rset, err)
