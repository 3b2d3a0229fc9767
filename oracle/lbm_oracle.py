"""FP64 reference implementation ("the oracle") of the D3Q19 MRT permeability solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It is deliberately
plain and slow: a dense periodic grid, a pull-scheme stream done with
``torch.roll``, an explicit 19x19 moment matrix applied by matrix products,
FP64 throughout.  It shares no code with the HIP implementation.

What it computes (all citations are to Rao & Schaefer, "Lattice Boltzmann
Models for Micro-tomographic Pore-spaces", arXiv:1902.11193):

* the lattice Boltzmann equation, stream + collide + force (Sec. 2, Eq. LBE);
* the D3Q19 lattice (Sec. 2); the weights are not printed in the paper and are
  the standard ones (1/3, 1/18, 1/36);
* MRT collision in moment space, C = -M^-1 S (m - m_eq) (Sec. 2.1.1,
  Eqs. MRT Collision / momentTransformation / LBE-MRT), with the moment order
  (rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz,
  mx, my, mz) and the rows of M from d'Humieres et al. (2002), whose polynomial
  definitions are written out in ``moment_matrix``;
* the equilibrium moments of Eq. MRT Equi, incompressible form (quadratic
  terms divided by rho0), with three misprints read as corrected: m1_eq has
  -11 rho, m9_eq is (2jx^2 - jy^2 - jz^2)/rho0, and m10_eq, m12_eq are -1/2 of
  m9_eq, m11_eq;
* the relaxation matrix S (Eq. MRT params) with the rate sets SRT, A-E of
  Table 2 and the magic parameter Lambda (Eq. Magic param);
* Guo body forcing in MRT (Eq. MRT-LBE, Eq. Guo_Forcing and the
  post-collision moments that follow it): the source F_i is built from the
  shifted velocity u = (sum_i f_i c_i + F/2)/rho0 and projected with M;
* halfway bounce-back at solid voxels (Sec. 2.3, the wall midway between a
  fluid and a solid voxel) in a periodic box with a body force (Sec. 2.3);
  as options, the paper's full-way bounce-back and symmetry (mirror) planes
  on the box faces (Sec. 2.3), and Zou-He pressure boundaries on the x faces
  with k from the pressure drop (Sec. 2.3, 3.1, Eq. perm_calc);
* the two-relaxation-time collision in velocity space (Sec. 2.1.2), the
  link-wise form of the MRT collision for two-rate sets (SRT, B, E);
* the Darcy permeability k_j = nu <u_j> / g_j from the volume-averaged
  velocity (Sec. 3, Eq. perm_calc) and the per-step convergence test
  (Eq. convergence).

Readings where the paper is silent or ambiguous: rho0 = 1; the velocity in
k is the shifted one; the volume average divides by all voxels (fluid and
solid); the state starts at rest, f_i = w_i rho0; step n is gather, then
collide, and <u>_n is taken from the distributions gathered at step n.

The gradient routine differentiates the same forward map with PyTorch's
reverse-mode autograd (segment-wise recomputation), so it is the exact
discrete adjoint of this oracle at FP64.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import torch

DT = torch.float64
RHO0 = 1.0

SETS = ("SRT", "A", "B", "C", "D", "E")


# --------------------------------------------------------------------------
# Lattice (Sec. 2)
# --------------------------------------------------------------------------
def velocities() -> torch.Tensor:
    """The 19 D3Q19 velocities as an int64 (19, 3) tensor, columns (cx, cy, cz).

    All c in {-1,0,1}^3 with |c|^2 <= 2: the rest vector, 6 face and 12 edge
    neighbours.  The order (by |c|^2, then lexicographic) is this module's own.
    """
    cs = [c for c in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in c) <= 2]
    cs.sort(key=lambda c: (sum(a * a for a in c), c))
    return torch.tensor(cs, dtype=torch.int64)


def weights(c: torch.Tensor) -> torch.Tensor:
    """Lattice weights: 1/3 (rest), 1/18 (|c|^2 = 1), 1/36 (|c|^2 = 2)."""
    q = (c * c).sum(1)
    w = torch.empty(len(c), dtype=DT)
    w[q == 0] = 1.0 / 3.0
    w[q == 1] = 1.0 / 18.0
    w[q == 2] = 1.0 / 36.0
    return w


def opposite(c: torch.Tensor) -> torch.Tensor:
    """Index of -c_i for every i."""
    lut = {tuple(v.tolist()): i for i, v in enumerate(c)}
    return torch.tensor([lut[tuple((-v).tolist())] for v in c], dtype=torch.int64)


# --------------------------------------------------------------------------
# Moment space (Sec. 2.1.1)
# --------------------------------------------------------------------------
MOMENT_NAMES = ("rho", "e", "eps", "jx", "qx", "jy", "qy", "jz", "qz",
                "3pxx", "3pixx", "pww", "piww", "pxy", "pyz", "pxz", "mx", "my", "mz")


def moment_matrix(c: torch.Tensor) -> torch.Tensor:
    """The 19x19 transformation matrix M (Eq. momentTransformation).

    Row k evaluates the k-th basis polynomial of d'Humieres et al. (2002) at
    every velocity, in the paper's moment order; q = |c|^2.
    """
    cx, cy, cz = (c[:, a].to(DT) for a in range(3))
    q = cx * cx + cy * cy + cz * cz
    one = torch.ones_like(cx)
    rows = [
        one,                                   # rho
        19 * q - 30,                           # e
        (21 * q * q - 53 * q + 24) / 2,        # epsilon
        cx, (5 * q - 9) * cx,                  # jx, qx
        cy, (5 * q - 9) * cy,                  # jy, qy
        cz, (5 * q - 9) * cz,                  # jz, qz
        3 * cx * cx - q,                       # 3 pxx
        (3 * q - 5) * (3 * cx * cx - q),       # 3 pixx
        cy * cy - cz * cz,                     # pww
        (3 * q - 5) * (cy * cy - cz * cz),     # piww
        cx * cy, cy * cz, cx * cz,             # pxy, pyz, pxz
        (cy * cy - cz * cz) * cx,              # mx
        (cz * cz - cx * cx) * cy,              # my
        (cx * cx - cy * cy) * cz,              # mz
    ]
    return torch.stack(rows)


def equilibrium_moments(rho: torch.Tensor, j: torch.Tensor, linear: bool = False) -> torch.Tensor:
    """Equilibrium moments m_eq(rho, j) of Eq. MRT Equi (incompressible form).

    ``rho``: (N,), ``j``: (3, N) shifted momentum.  With ``linear`` the
    quadratic terms are dropped (the Stokes simplification the paper mentions
    after Eq. MRT params, used here only for exact invariants).
    """
    jx, jy, jz = j
    z = torch.zeros_like(rho)
    if linear:
        jj = xx = yy = zz = xy = yz = xz = z
    else:
        xx, yy, zz = jx * jx / RHO0, jy * jy / RHO0, jz * jz / RHO0
        jj = xx + yy + zz
        xy, yz, xz = jx * jy / RHO0, jy * jz / RHO0, jx * jz / RHO0
    m9 = 2 * xx - yy - zz
    m11 = yy - zz
    return torch.stack([
        rho,
        -11 * rho + 19 * jj,
        3 * rho - 5.5 * jj,
        jx, -2.0 / 3.0 * jx,
        jy, -2.0 / 3.0 * jy,
        jz, -2.0 / 3.0 * jz,
        m9, -0.5 * m9,
        m11, -0.5 * m11,
        xy, yz, xz,
        z, z, z,
    ])


def guo_source(c: torch.Tensor, w: torch.Tensor, u: torch.Tensor, F: torch.Tensor,
               linear: bool = False) -> torch.Tensor:
    """Guo forcing term F_i (Eq. Guo_Forcing) with c_s^2 = 1/3.

    F_i = w_i [ 3 (c_i - u) . F + 9 (c_i . u)(c_i . F) ];  u, F: (3, N).
    ``linear`` keeps only the term linear in the small quantities, 3 w_i c_i.F.
    """
    cf = c.to(DT)
    cF = cf @ F                      # (19, N)
    if linear:
        return 3.0 * w[:, None] * cF
    cu = cf @ u
    uF = (u * F).sum(0)[None, :]
    return w[:, None] * (3.0 * (cF - uF) + 9.0 * cu * cF)


# --------------------------------------------------------------------------
# Relaxation rates (Table 2, Eq. Magic param)
# --------------------------------------------------------------------------
def rates(rset: str, tau, Lambda=None) -> torch.Tensor:
    """The 19 diagonal entries of S for a relaxation set of Table 2.

    ``tau`` and ``Lambda`` may be Python floats or 0-d float64 tensors (the
    result is then differentiable in them).  s_nu = 1/tau drives moments 9, 11,
    13, 14, 15 in every set; rho, jx, jy, jz have rate 0.  Set E keeps
    Lambda = (1/s+ - 1/2)(1/s- - 1/2) fixed (Eq. Magic param) by
    s- = 2 (2 - s_nu) / (4 Lambda s_nu - s_nu + 2).
    """
    tau = torch.as_tensor(tau, dtype=DT)
    if not float(tau.detach()) > 0.5:
        raise ValueError("tau must exceed 1/2")
    s = 1.0 / tau
    a = 8 * (2 - s) / (8 - s)
    b = 4 * (2 - s) / (4 + s)
    if rset == "SRT":
        se = seps = sq = spi = sm = s
    elif rset == "A":
        se = seps = sq = spi = sm = a
    elif rset == "B":
        se = seps = spi = s
        sq = sm = a
    elif rset == "C":
        se, seps, sq, spi, sm = (torch.tensor(v, dtype=DT) for v in (1.19, 1.4, 1.2, 1.4, 1.98))
    elif rset == "D":
        se = seps = spi = s
        sq, sm = a, b
    elif rset == "E":
        if Lambda is None:
            raise ValueError("Set E needs Lambda")
        Lam = torch.as_tensor(Lambda, dtype=DT)
        if not float(Lam.detach()) > 0:
            raise ValueError("Lambda must be positive")
        se = seps = spi = s
        sq = sm = 2 * (2 - s) / (4 * Lam * s - s + 2)
    else:
        raise ValueError(f"unknown relaxation set {rset!r}")
    zero = torch.zeros((), dtype=DT)
    out = torch.stack([zero, se, seps, zero, sq, zero, sq, zero, sq,
                       s, spi, s, spi, s, s, s, sm, sm, sm])
    nz = out[[1, 2, 4, 6, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18]]
    if not bool(((nz > 0) & (nz < 2)).all()):
        raise ValueError("every non-conserved rate must lie in (0, 2)")
    return out


def viscosity(tau) -> float:
    """nu = c_s^2 (tau - 1/2) with c_s^2 = 1/3 (Sec. 2.1)."""
    return (tau - 0.5) / 3.0


# --------------------------------------------------------------------------
# One time step
# --------------------------------------------------------------------------
@dataclass
class Lattice:
    c: torch.Tensor
    w: torch.Tensor
    opp: torch.Tensor
    M: torch.Tensor
    Minv: torch.Tensor

    @staticmethod
    def make() -> "Lattice":
        c = velocities()
        M = moment_matrix(c)
        return Lattice(c, weights(c), opposite(c), M, torch.linalg.inv(M))


def stream(fh: torch.Tensor, solid: torch.Tensor, lat: Lattice) -> torch.Tensor:
    """Pull streaming with halfway bounce-back on a periodic grid.

    ``fh``: post-collision populations (19, nz, ny, nx).  The incoming
    f_i(x) is fh_i(x - c_i); when x - c_i is a solid voxel the population
    that left x towards the wall returns reversed, f_i(x) = fh_ibar(x).
    """
    out = torch.empty_like(fh)
    for i in range(19):
        cx, cy, cz = (int(v) for v in lat.c[i])
        sh = (cz, cy, cx)
        pulled = torch.roll(fh[i], shifts=sh, dims=(0, 1, 2))
        from_solid = torch.roll(solid, shifts=sh, dims=(0, 1, 2))
        out[i] = torch.where(from_solid, fh[int(lat.opp[i])], pulled)
    return out


def mirror(i: int, axis: int, lat: Lattice) -> int:
    """Index of the velocity c_i reflected in ``axis`` (0 = x, 1 = y, 2 = z)."""
    c = lat.c[i].clone()
    c[axis] = -c[axis]
    return int(torch.nonzero((lat.c == c).all(1))[0])


def stream_general(fh: torch.Tensor, solid: torch.Tensor, lat: Lattice, symmetric=(False, False, False),
                   fh_wall: torch.Tensor | None = None) -> torch.Tensor:
    """Pull streaming written out voxel by voxel (index arrays), with two
    options the periodic ``stream`` lacks:

    * ``symmetric[a]``: the box faces normal to axis a are symmetry (mirror)
      planes, half a voxel outside the first and last layers (Sec. 2.3): a pull
      that leaves the box through such a face takes, from the voxel reached by
      the tangential part of the step alone, the population of the velocity
      mirrored in that axis;
    * ``fh_wall``: the state the bounce-back reads, fh itself for halfway
      bounce-back, or the state one step older for full-way bounce-back, where
      a population reaches the wall voxel, turns there at the next collision
      and comes back one step later than with the wall midway (Sec. 2.3).

    Halfway bounce-back applies when the (mirrored) source voxel is solid.
    """
    nz, ny, nx = solid.shape
    n = (nx, ny, nz)
    wall_state = fh if fh_wall is None else fh_wall
    z, y, x = torch.meshgrid(torch.arange(nz), torch.arange(ny), torch.arange(nx), indexing="ij")
    coord = (x, y, z)
    mtab = [torch.tensor([mirror(p, a, lat) for p in range(19)]) for a in range(3)]
    out = torch.empty_like(fh)
    for i in range(19):
        src = [coord[a] - int(lat.c[i][a]) for a in range(3)]
        pop = torch.full(solid.shape, i, dtype=torch.long)
        for a in range(3):
            if symmetric[a]:
                # |c_a| <= 1: a pull that leaves the box comes from the voxel
                # itself in axis a, with the velocity mirrored in that axis
                leaves = (src[a] < 0) | (src[a] >= n[a])
                src[a] = torch.where(leaves, coord[a], src[a])
                pop = torch.where(leaves, mtab[a][pop], pop)
            src[a] = src[a] % n[a]
        from_solid = solid[src[2], src[1], src[0]]
        pulled = fh[pop, src[2], src[1], src[0]]
        bounced = wall_state[int(lat.opp[i])]
        out[i] = torch.where(from_solid, bounced, pulled)
    return out


def zou_he_pressure(f: torch.Tensor, lat: Lattice, rho_in: float, rho_out: float) -> torch.Tensor:
    """Zou-He pressure boundaries on the x faces (Sec. 2.3, Sec. 3.1): at the
    fluid voxels of the plane x = 0 the five populations with c_x = +1, and of
    x = nx - 1 those with c_x = -1, come from outside the image; they are
    rebuilt so that the density is the prescribed one, the transverse velocity
    is zero, and the non-equilibrium parts of opposite populations along x
    are equal, with the transverse momentum of the known populations cancelled
    on the diagonals.  ``f``: gathered populations (19, nz, ny, nx), full
    (not deviations), changed in place and returned."""
    c = lat.c
    cx = c[:, 0]
    for plane, rho_b, sgn in ((0, rho_in, 1), (f.shape[-1] - 1, rho_out, -1)):
        g = f[..., plane]                                   # (19, nz, ny)
        known0 = [i for i in range(19) if cx[i] == 0]
        back = [i for i in range(19) if cx[i] == -sgn]      # leaving the box through this face
        ju = sgn * (rho_b - g[known0].sum(0) - 2.0 * g[back].sum(0))   # rho u_x, sign of x
        ny_ = 0.5 * sum(float(c[i, 1]) * g[i] for i in known0)
        nz_ = 0.5 * sum(float(c[i, 2]) * g[i] for i in known0)
        for i in range(19):
            if cx[i] != sgn:
                continue
            b = int(lat.opp[i])
            cy, cz = float(c[i, 1]), float(c[i, 2])
            if cy == 0 and cz == 0:
                g[i] = g[b] + sgn * ju / 3.0
            else:
                # w = 1/36 diagonal: rho (c.u)/6 with u = (u_x, 0, 0), minus the
                # transverse momentum of the in-plane populations
                g[i] = g[b] + sgn * ju / 6.0 - cy * ny_ - cz * nz_
        f[..., plane] = g
    return f


def macroscopic(f: torch.Tensor, F: torch.Tensor, lat: Lattice):
    """rho = sum f, shifted momentum j = sum f c + F/2, u = j / rho0."""
    m = lat.M @ f
    rho = m[0]
    j = m[[3, 5, 7]] + 0.5 * F
    return m, rho, j, j / RHO0


def collide(f: torch.Tensor, s: torch.Tensor, F: torch.Tensor, lat: Lattice,
            linear: bool = False) -> torch.Tensor:
    """MRT collision with Guo forcing at fluid nodes; ``f``: (19, N), ``F``: (3, N).

    m* = m - S (m - m_eq) + (I - S/2) M F_i, then f* = M^-1 m*.
    """
    m, rho, j, u = macroscopic(f, F, lat)
    meq = equilibrium_moments(rho, j, linear)
    mF = lat.M @ guo_source(lat.c, lat.w, u, F, linear)
    S = s[:, None]
    mstar = m - S * (m - meq) + (1.0 - 0.5 * S) * mF
    return lat.Minv @ mstar


# --------------------------------------------------------------------------
# Two-relaxation-time collision in velocity space (Sec. 2.1.2)
# --------------------------------------------------------------------------
EVEN_ROWS = [1, 2, 9, 10, 11, 12, 13, 14, 15]   # e, eps, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz
ODD_ROWS = [4, 6, 8, 16, 17, 18]                 # qx, qy, qz, mx, my, mz


def trt_rates(s: torch.Tensor):
    """(s+, s-) of a rate vector that is a two-relaxation-time set: every
    non-conserved even moment relaxes at s+ and every odd one at s- (SRT, Set B
    and Set E of Table 2 are; Sets A, C and D are not)."""
    even, odd = s[EVEN_ROWS], s[ODD_ROWS]
    if not (bool((even == even[0]).all()) and bool((odd == odd[0]).all())):
        raise ValueError("the rates are not a two-relaxation-time set")
    return even[0], odd[0]


def equilibrium(c: torch.Tensor, w: torch.Tensor, rho: torch.Tensor, j: torch.Tensor,
                linear: bool = False) -> torch.Tensor:
    """Incompressible second-order equilibrium in velocity space, rho0 = 1:
    f_eq,i = w_i [rho + 3 c_i.j + 9/2 (c_i.j)^2 - 3/2 j.j]; ``linear`` drops the
    quadratic terms.  Its moments are the m_eq of Eq. MRT Equi as read here."""
    cj = c.to(DT) @ j
    out = rho[None, :] + 3.0 * cj
    if not linear:
        out = out + (4.5 * cj * cj - 1.5 * (j * j).sum(0)[None, :]) / RHO0
    return w[:, None] * out


def collide_trt(f: torch.Tensor, s: torch.Tensor, F: torch.Tensor, lat: Lattice,
                linear: bool = False) -> torch.Tensor:
    """Link-wise TRT collision with Guo forcing; ``f``: (19, N), ``F``: (3, N).

    Each population and its opposite split into a symmetric part
    (f_i + f_ibar)/2 and an antisymmetric part (f_i - f_ibar)/2.  The symmetric
    parts relax towards those of f_eq at s+ and gain (1 - s+/2) times those of
    Guo's F_i; the antisymmetric parts do the same with s-.  With j the shifted
    momentum in f_eq this is the MRT collision of a two-rate set: the
    momentum, which MRT leaves unrelaxed, gains s- F/2 from the relaxation
    towards f_eq(j) and (1 - s-/2) F from the source, F in all.
    """
    sp, sm = trt_rates(s)
    opp = lat.opp
    rho = f.sum(0)
    j = lat.c.to(DT).T @ f + 0.5 * F
    feq = equilibrium(lat.c, lat.w, rho, j, linear)
    Fi = guo_source(lat.c, lat.w, j / RHO0, F, linear)
    sym = lambda a: 0.5 * (a + a[opp])
    anti = lambda a: 0.5 * (a - a[opp])
    return (f - sp * (sym(f) - sym(feq)) - sm * (anti(f) - anti(feq))
            + (1.0 - 0.5 * sp) * sym(Fi) + (1.0 - 0.5 * sm) * anti(Fi))


def rest_state(fluid: torch.Tensor, lat: Lattice) -> torch.Tensor:
    """Initial state f_i = w_i rho0 at fluid voxels, 0 in solid."""
    return lat.w[:, None, None, None] * RHO0 * fluid.to(DT)[None]


class Problem:
    """A voxel image with its parameters; dense FP64 state on the CPU."""

    def __init__(self, mask: np.ndarray, tau: float, Lambda: float | None, rset: str,
                 g, g_field: np.ndarray | None = None, linear: bool = False, collision: str = "mrt",
                 symmetric: str = "", fullway: bool = False, pressure=None):
        self.lat = Lattice.make()
        # Zou-He pressure boundaries on the x faces, (rho_in, rho_out): the box
        # is then not periodic in x and k follows from the pressure drop
        self.pressure = None if pressure is None else (float(pressure[0]), float(pressure[1]))
        # symmetry planes on the faces normal to the named axes (subset of "xyz"),
        # and full-way instead of halfway bounce-back (Sec. 2.3)
        self.symmetric = tuple(a in symmetric for a in "xyz")
        self.fullway = bool(fullway)
        self.general = any(self.symmetric) or self.fullway or self.pressure is not None
        if collision not in ("mrt", "trt"):
            raise ValueError("collision must be 'mrt' or 'trt'")
        self.collision = collision
        mask = np.asarray(mask)
        self.shape = mask.shape
        self.solid = torch.from_numpy(mask != 0)
        self.fluid = ~self.solid
        self.nf = int(self.fluid.sum())
        if self.nf == 0:
            raise ValueError("no fluid voxels")
        self.volume = float(mask.size)
        self.tau = float(tau)
        self.Lambda = None if Lambda is None else float(Lambda)
        self.rset = rset
        self.g = torch.as_tensor(np.asarray(g, dtype=np.float64))
        self.linear = linear
        if g_field is None:
            gf = self.g[:, None].expand(3, self.nf)
        else:
            gf = torch.from_numpy(np.asarray(g_field, dtype=np.float64))[:, self.fluid]
        self.F = RHO0 * gf.clone()          # force density at fluid voxels, (3, N_f)
        self.s = rates(rset, self.tau, self.Lambda)
        if collision == "trt":
            trt_rates(self.s)
        self.nu = viscosity(self.tau)

    def initial(self) -> torch.Tensor:
        """fh at rest; with full-way bounce-back the state also carries the
        previous step's fh (stacked: [this step, one step older])."""
        r = rest_state(self.fluid, self.lat)
        return torch.stack([r, r.clone()]) if self.fullway else r

    def step(self, fh: torch.Tensor, s=None, F=None):
        """One step: gather, then collide.  Returns (new fh, u of this step)."""
        s = self.s if s is None else s
        F = self.F if F is None else F
        if self.fullway:
            new, u = self._step(fh[0], s, F, fh_wall=fh[1])
            return torch.stack([new, fh[0]]), u
        return self._step(fh, s, F)

    def _step(self, fh, s, F, fh_wall=None):
        if self.general:
            f = stream_general(fh, self.solid, self.lat, self.symmetric, fh_wall)
            if self.pressure is not None:
                f = zou_he_pressure(f, self.lat, *self.pressure) * self.fluid.to(DT)[None]
        else:
            f = stream(fh, self.solid, self.lat)
        ff = f[:, self.fluid]
        out = torch.zeros_like(fh)
        col = collide_trt if self.collision == "trt" else collide
        out[:, self.fluid] = col(ff, s, F, self.lat, self.linear)
        _, _, _, u = macroscopic(ff, F, self.lat)
        return out, u

    def mean_velocity(self, u: torch.Tensor) -> torch.Tensor:
        """Superficial volume average: sum over fluid / all voxels (Eq. perm_calc)."""
        return u.sum(1) / self.volume

    def permeability(self, umean: torch.Tensor) -> torch.Tensor:
        """k_j = nu <u_j> / g_j (Eq. perm_calc with the pressure gradient dropped);
        with pressure boundaries k_x = nu <u_x> / grad p, grad p = c_s^2 (rho_in -
        rho_out) / (nx - 1) between the boundary planes (Eq. perm_calc, rho0 = 1)."""
        if self.pressure is not None:
            gp = (self.pressure[0] - self.pressure[1]) / 3.0 / (self.shape[-1] - 1)
            out = torch.full_like(umean, float("nan"))
            out[0] = self.nu * umean[0] / gp
            return out
        return torch.where(self.g != 0, self.nu * umean / self.g,
                           torch.full_like(umean, float("nan")))


def run(problem: Problem, n_steps: int, keep_state: bool = True):
    """March ``n_steps`` steps from rest.  Returns dict with the per-step mean
    velocity history (n_steps, 3), the final k, and the final state."""
    fh = problem.initial()
    hist = torch.empty((n_steps, 3), dtype=DT)
    for n in range(n_steps):
        fh, u = problem.step(fh)
        hist[n] = problem.mean_velocity(u)
    k = problem.permeability(hist[-1]) if n_steps else None
    return dict(umean=hist, k=k, state=fh if keep_state else None)


def run_to_steady(problem: Problem, eps: float, max_steps: int, min_steps: int = 2):
    """Step until |k_n - k_(n-1)| / |k_n| < eps in the driven direction (Eq. convergence)."""
    axis = int(torch.argmax(problem.g.abs()))
    fh = problem.initial()
    prev = None
    k = None
    for n in range(1, max_steps + 1):
        fh, u = problem.step(fh)
        k = problem.permeability(problem.mean_velocity(u))
        kn = float(k[axis])
        if prev is not None and n >= min_steps and abs(kn - prev) < eps * abs(kn):
            return dict(steps=n, k=k, state=fh, converged=True)
        prev = kn
    return dict(steps=max_steps, k=k, state=fh, converged=False)


def state_at_fluid(problem: Problem, fh: torch.Tensor) -> torch.Tensor:
    """Post-collision populations at fluid voxels in raster order (x fastest): (19, N_f)."""
    return fh[:, problem.fluid]


# --------------------------------------------------------------------------
# Gradients: reverse-mode through the same forward map
# --------------------------------------------------------------------------
def gradients(problem: Problem, n_steps: int, segment: int = 50):
    """k_N along the driving axis and its exact derivatives at step N.

    Returns dict(k, dk_dtau, dk_dLambda, dk_dg) where dk_dg is (3, N_f): the
    derivative with respect to the body-force acceleration at each fluid voxel
    (raster order), with the normalising g in k = nu <u> / g held at the value
    the problem was built with.  The forward is recomputed segment by segment
    (``segment`` steps each) so memory stays bounded.
    """
    if problem.general:
        raise NotImplementedError("gradients are for the periodic halfway bounce-back problem")
    axis = int(torch.argmax(problem.g.abs()))
    gref = float(problem.g[axis])
    tau_t = torch.tensor(problem.tau, dtype=DT, requires_grad=True)
    lam0 = problem.Lambda if problem.Lambda is not None else 0.25
    lam_t = torch.tensor(lam0, dtype=DT, requires_grad=True)
    F_t = problem.F.clone().requires_grad_(True)

    def rates_t():
        return rates(problem.rset, tau_t, lam_t if problem.rset == "E" else None)

    def advance(fh, nsteps):
        s = rates_t()
        for _ in range(nsteps):
            fh, _ = problem.step(fh, s=s, F=F_t)
        return fh

    def readout(fh):
        f = stream(fh, problem.solid, problem.lat)
        ff = f[:, problem.fluid]
        _, _, _, u = macroscopic(ff, F_t, problem.lat)
        nu = (tau_t - 0.5) / 3.0
        return nu * u[axis].sum() / problem.volume / gref

    # forward pass, keeping segment-start snapshots of fh^0 ... fh^(N-1)
    nfw = n_steps - 1
    bounds = list(range(0, nfw, segment)) + [nfw]
    snaps = []
    fh = problem.initial()
    with torch.no_grad():
        for a, b in zip(bounds[:-1], bounds[1:]):
            snaps.append(fh.clone())
            fh = advance(fh, b - a)
    last = fh.detach().requires_grad_(True)
    k = readout(last)
    g_tau, g_lam, g_F, adj = torch.autograd.grad(k, [tau_t, lam_t, F_t, last], allow_unused=True)
    g_tau = g_tau if g_tau is not None else torch.zeros((), dtype=DT)
    g_lam = g_lam if g_lam is not None else torch.zeros((), dtype=DT)
    g_F = g_F if g_F is not None else torch.zeros_like(F_t)
    for (a, b), snap in zip(reversed(list(zip(bounds[:-1], bounds[1:]))), reversed(snaps)):
        x0 = snap.clone().requires_grad_(True)
        out = advance(x0, b - a)
        gt, gl, gF, adj = torch.autograd.grad(out, [tau_t, lam_t, F_t, x0], grad_outputs=adj,
                                              allow_unused=True)
        if gt is not None:
            g_tau = g_tau + gt
        if gl is not None:
            g_lam = g_lam + gl
        if gF is not None:
            g_F = g_F + gF
    if problem.rset != "E":
        g_lam = torch.zeros((), dtype=DT)
    return dict(k=float(k), dk_dtau=float(g_tau), dk_dLambda=float(g_lam),
                dk_dg=(g_F * RHO0).detach())


# --------------------------------------------------------------------------
# Helpers for comparisons
# --------------------------------------------------------------------------
def unit_darcy(k_lu: float, dx_m: float) -> float:
    """Lattice permeability to darcy: k_lu dx^2 / 0.9869e-12 m^2 (Sec. 3.3, read as corrected)."""
    return k_lu * dx_m * dx_m / 0.9869233e-12


def time_steps(problem: Problem, n_steps: int) -> float:
    """Wall seconds for ``n_steps`` oracle steps from rest (CPU baseline timing)."""
    import time
    fh = problem.initial()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        fh, _ = problem.step(fh)
    return time.perf_counter() - t0


__all__ = [
    "velocities", "weights", "opposite", "moment_matrix", "equilibrium_moments", "guo_source",
    "rates", "viscosity", "Lattice", "stream", "macroscopic", "collide", "rest_state",
    "Problem", "run", "run_to_steady", "state_at_fluid", "gradients", "unit_darcy",
    "time_steps", "SETS", "MOMENT_NAMES", "RHO0", "trt_rates", "equilibrium", "collide_trt",
    "EVEN_ROWS", "ODD_ROWS", "mirror", "stream_general", "zou_he_pressure",
]
