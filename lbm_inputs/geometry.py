"""Synthetic segmented voxel images (0 = fluid, 1 = solid), periodic boxes.

Every array is ``uint8[nz][ny][nx]`` with x the fastest axis, the layout the
C-ABI takes.  Generators are seeded (``numpy.random.default_rng``) so the same
call returns the same image on every machine.

The shapes mirror the paper's test geometries (Sec. 3: circular and
triangular channels, random sphere packs; Sec. 1/2: segmented micro-CT
rock), synthesised here because the paper's image stacks are not available.
"""
from __future__ import annotations

import math

import numpy as np

FLUID = 0
SOLID = 1


def porosity(mask: np.ndarray) -> float:
    """Fraction of fluid voxels."""
    return float(np.count_nonzero(mask == FLUID)) / mask.size


def _grid(n: tuple[int, int, int]):
    nz, ny, nx = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z


def sphere(n: int, center=(15.5, 15.5, 15.5), radius: float = 8.0) -> np.ndarray:
    """One solid ball in a periodic ``n**3`` box: a simple-cubic sphere array.

    A voxel (centre at integer coordinates) is solid iff its minimum-image
    squared distance to ``center`` is <= ``radius**2``.
    """
    x, y, z = _grid((n, n, n))
    cx, cy, cz = center

    def d(a, c):
        t = np.abs(a - c)
        return np.minimum(t, n - t)

    r2 = d(x, cx) ** 2 + d(y, cy) ** 2 + d(z, cz) ** 2
    return (r2 <= radius * radius).astype(np.uint8)


def slit(nx: int, ny: int, nz: int, h: int) -> np.ndarray:
    """Plane channel: rows ``y < h`` are fluid, the rest solid (walls normal to y)."""
    if not 0 < h < ny:
        raise ValueError("need 0 < h < ny")
    m = np.ones((nz, ny, nx), np.uint8)
    m[:, :h, :] = FLUID
    return m


def duct(nx: int, a: int, wall: int = 1) -> np.ndarray:
    """Square duct along x with an ``a x a`` fluid cross-section and ``wall`` solid layers."""
    n = a + wall
    m = np.ones((n, n, nx), np.uint8)
    m[:a, :a, :] = FLUID
    return m


def pipe(nx: int, n: int, radius: float) -> np.ndarray:
    """Circular channel along x in an ``n x n`` cross-section (fluid iff r < radius).

    The paper's first test geometry (Sec. 3.1, Eq. for k of a circular bore).
    """
    c = (n - 1) / 2.0
    y, z = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    r2 = (y - c) ** 2 + (z - c) ** 2
    sec = np.where(r2 < radius * radius, FLUID, SOLID).astype(np.uint8)
    return np.ascontiguousarray(np.broadcast_to(sec[:, :, None], (n, n, nx)))


def triangle_channel(nx: int, n: int, side: float) -> np.ndarray:
    """Channel along x with an equilateral-triangle cross-section of the given side.

    The paper's second test geometry (Sec. 3.2).  Voxel centres strictly inside
    the triangle are fluid.
    """
    c = (n - 1) / 2.0
    hgt = side * math.sqrt(3.0) / 2.0
    y0 = c - hgt / 3.0  # base line (centroid at c)
    yy, zz = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="xy")
    # z is the in-plane horizontal coordinate, y the vertical one
    inside = (yy > y0) & (yy < y0 + hgt)
    half = (y0 + hgt - yy) / math.sqrt(3.0)
    inside &= np.abs(zz - c) < half
    sec = np.where(inside.T, FLUID, SOLID).astype(np.uint8)  # [z][y]
    return np.ascontiguousarray(np.broadcast_to(sec[:, :, None], (n, n, nx)))


def _stamp_ball(solid: np.ndarray, c: np.ndarray, radius: float) -> None:
    """Mark voxels within ``radius`` of ``c`` (periodic) as solid, in place."""
    nz, ny, nx = solid.shape
    r = int(math.ceil(radius))
    off = np.arange(-r, r + 1)
    oz, oy, ox = np.meshgrid(off, off, off, indexing="ij")
    base = np.floor(c).astype(int)
    px = base[0] + ox
    py = base[1] + oy
    pz = base[2] + oz
    d2 = (px - c[0]) ** 2 + (py - c[1]) ** 2 + (pz - c[2]) ** 2
    sel = d2 <= radius * radius
    solid[pz[sel] % nz, py[sel] % ny, px[sel] % nx] = 1


def sphere_pack(n: int, radius: float, target_porosity: float, seed: int,
                hard_core: float | None = None) -> np.ndarray:
    """Random pack of equal solid balls by seeded random sequential addition.

    Centres are drawn uniformly in the periodic box and accepted when they are
    at least ``2 * hard_core`` from every accepted centre; each accepted ball
    of ``radius`` is stamped, until the porosity falls to ``target_porosity``.
    Non-overlapping addition (``hard_core == radius``) jams near a solid
    fraction of 0.38, so lower targets need a smaller hard core; when the
    addition jams (2000 rejections in a row) the hard core shrinks by 5 %
    and addition continues.  This follows the paper's picture of a pack of
    identical spheres (Sec. 3.3) at the requested porosity.
    """
    rng = np.random.default_rng(seed)
    solid = np.zeros((n, n, n), np.uint8)
    hc = radius if hard_core is None else hard_core
    centres = np.zeros((0, 3))
    fails = 0
    nsolid_target = (1.0 - target_porosity) * solid.size
    while np.count_nonzero(solid) < nsolid_target:
        c = rng.uniform(0.0, n, size=3)
        if len(centres):
            d = np.abs(centres - c)
            d = np.minimum(d, n - d)
            if np.min(np.einsum("ij,ij->i", d, d)) < (2 * hc) ** 2:
                fails += 1
                if fails >= 2000:
                    hc *= 0.95
                    fails = 0
                continue
        fails = 0
        centres = np.vstack([centres, c])
        _stamp_ball(solid, c, radius)
    return solid


_D18 = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
        if 0 < dx * dx + dy * dy + dz * dz <= 2]


def percolating_x(mask: np.ndarray) -> np.ndarray:
    """Remove fluid that does not belong to an x-spanning cluster.

    Fluid voxels are linked to their 18 lattice neighbours (the D3Q19 links),
    periodically across the y and z faces but not across x.  Clusters that
    contain fluid in both the x = 0 and x = nx-1 planes span the sample from
    inlet to outlet and are kept; every other fluid voxel becomes solid.
    """
    import scipy.ndimage as ndi
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    fluid = mask == FLUID
    st = np.zeros((3, 3, 3), bool)
    for d in _D18:
        st[d[0] + 1, d[1] + 1, d[2] + 1] = True
    st[1, 1, 1] = True
    lab, nl = ndi.label(fluid, structure=st)
    if nl == 0:
        return np.ones_like(mask)
    nz, ny, nx = mask.shape
    pa, pb = [], []
    # links that cross the periodic z and y faces
    for d in _D18:
        dz, dy, dx = d
        for axis, dd, size in ((0, dz, nz), (1, dy, ny)):
            if dd != 1:
                continue
            src = np.take(lab, [size - 1], axis=axis)
            dst = np.take(lab, [0], axis=axis)
            # shift the destination plane by the in-plane offsets (periodic in the
            # other periodic axis, open in x)
            sh = [0, 0, 0]
            if axis == 0:
                sh[1] = dy
            else:
                sh[0] = dz
            dst = np.roll(dst, shift=(-sh[0], -sh[1]), axis=(0, 1))
            if dx != 0:
                t = np.zeros_like(dst)
                if dx == 1:
                    t[..., :-1] = dst[..., 1:]
                else:
                    t[..., 1:] = dst[..., :-1]
                dst = t
            sel = (src > 0) & (dst > 0) & (src != dst)
            pa.append(src[sel])
            pb.append(dst[sel])
    a = np.concatenate(pa) if pa else np.zeros(0, np.int64)
    b = np.concatenate(pb) if pb else np.zeros(0, np.int64)
    g = coo_matrix((np.ones(len(a)), (a, b)), shape=(nl + 1, nl + 1))
    _, comp = connected_components(g, directed=False)
    cl = comp[lab]
    left = np.unique(cl[:, :, 0][lab[:, :, 0] > 0])
    right = np.unique(cl[:, :, nx - 1][lab[:, :, nx - 1] > 0])
    keep = np.intersect1d(left, right)
    out = np.ones_like(mask)
    out[fluid & np.isin(cl, keep)] = FLUID
    return out


def _progress(msg: str, verbose: bool):
    if verbose:
        import sys
        print(f"[inputs] {msg}", file=sys.stderr, flush=True)


def gaussian_random_field(n: int, corr_len: float, target_porosity: float, seed: int,
                          filter_percolation: bool = True, verbose: bool = False) -> np.ndarray:
    """Thresholded Gaussian random field: a synthetic segmented rock image.

    White noise N(0, 1) is smoothed with a periodic Gaussian filter of standard
    deviation ``corr_len / sqrt(2)``, giving a field whose covariance decays as
    exp(-r^2 / (2 corr_len^2)).  The lowest ``target_porosity`` fraction of
    values becomes fluid (ties broken by linear index), then non-spanning
    fluid is removed (``percolating_x``).
    """
    import scipy.ndimage as ndi

    rng = np.random.default_rng(seed)
    field = rng.standard_normal((n, n, n), dtype=np.float32)
    # the separable Gaussian filter, one axis at a time (what gaussian_filter does)
    for axis in range(3):
        field = ndi.gaussian_filter1d(field, sigma=corr_len / math.sqrt(2.0), axis=axis, mode="wrap")
        _progress(f"grf {n}^3: filtered axis {axis}", verbose)
    flat = field.reshape(-1)
    nf = int(round(target_porosity * flat.size))
    thr = np.partition(flat, nf)[nf] if nf < flat.size else np.inf
    fluid = flat < thr
    short = nf - int(np.count_nonzero(fluid))
    if short > 0:
        ties = np.flatnonzero(flat == thr)[:short]
        fluid[ties] = True
    m = np.where(fluid, FLUID, SOLID).astype(np.uint8).reshape(n, n, n)
    del field, flat, fluid
    _progress(f"grf {n}^3: thresholded", verbose)
    if filter_percolation:
        m = percolating_x(m)
        _progress(f"grf {n}^3: percolation filter done", verbose)
    return m


def crop(mask: np.ndarray, size: int, origin=(0, 0, 0), filter_percolation: bool = True) -> np.ndarray:
    """A ``size**3`` sub-block (treated as a new periodic box), optionally re-filtered."""
    z0, y0, x0 = origin
    c = np.ascontiguousarray(mask[z0:z0 + size, y0:y0 + size, x0:x0 + size])
    if filter_percolation:
        c = percolating_x(c)
    return c


def random_mask(n: tuple[int, int, int], solid_fraction: float, seed: int) -> np.ndarray:
    """Independent Bernoulli voxels: a worst case for index tables and bounce-back."""
    rng = np.random.default_rng(seed)
    return (rng.random(n) < solid_fraction).astype(np.uint8)


# The five workloads the implementation is measured and checked on.  Seeds are
# 1902 + index.  Porosities are of the generated image (fluid fraction).
WORKLOADS = {
    "sc_sphere_32": dict(kind="sphere", n=32, radius=8.0, tau=1.0, Lambda=3 / 16, g=1e-6),
    "pack_256": dict(kind="pack", n=256, radius=12.0, porosity=0.40, seed=1903, g=1e-6),
    "grf_512": dict(kind="grf", n=512, corr_len=6.0, porosity=0.20, seed=1904, g=1e-6),
    "pack_128": dict(kind="pack", n=128, radius=8.0, porosity=0.38, seed=1905, g=1e-6),
    "grf_1024": dict(kind="grf", n=1024, corr_len=4.0, porosity=0.15, seed=1906, g=1e-7),
}


def workload(name: str, n: int | None = None, verbose: bool = False) -> np.ndarray:
    """Generate a named workload image (optionally at another edge length ``n``)."""
    w = WORKLOADS[name]
    size = n or w["n"]
    if w["kind"] == "sphere":
        c = (size - 1) / 2.0
        return sphere(size, (c, c, c), w["radius"] * size / w["n"])
    if w["kind"] == "pack":
        m = sphere_pack(size, w["radius"], w["porosity"], w["seed"], hard_core=0.8 * w["radius"])
        return percolating_x(m)
    if w["kind"] == "grf":
        return gaussian_random_field(size, w["corr_len"], w["porosity"], w["seed"], verbose=verbose)
    raise KeyError(name)
