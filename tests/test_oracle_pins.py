"""Pins for the FP64 oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself:
lattice isotropy, printed values of the paper (tests/golden/paper_values.json),
closed-form solutions, conservation laws, a velocity-space BGK collision and a
loop-by-loop brute-force step written here independently.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
from lbm_inputs import slit, duct, sphere, random_mask, percolating_x

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
LAT = O.Lattice.make()
C = LAT.c.to(torch.float64)


# ---------------------------------------------------------------- lattice
def test_velocity_set_is_d3q19():
    c = LAT.c
    assert len({tuple(v.tolist()) for v in c}) == 19
    q = (c * c).sum(1)
    assert sorted(q.tolist()) == [0] + [1] * 6 + [2] * 12
    assert torch.equal(c[LAT.opp], -c)


def test_weights_isotropy():
    """Weights reproduce the Maxwellian moments up to 4th order with c_s^2 = 1/3."""
    w = LAT.w
    assert abs(float(w.sum()) - 1) < 1e-15
    d = torch.eye(3, dtype=torch.float64)
    second = torch.einsum("i,ia,ib->ab", w, C, C)
    assert torch.allclose(second, d / 3, atol=1e-15)
    third = torch.einsum("i,ia,ib,ic->abc", w, C, C, C)
    assert float(third.abs().max()) < 1e-15
    fourth = torch.einsum("i,ia,ib,ic,id->abcd", w, C, C, C, C)
    iso = (torch.einsum("ab,cd->abcd", d, d) + torch.einsum("ac,bd->abcd", d, d)
           + torch.einsum("ad,bc->abcd", d, d)) / 9
    assert torch.allclose(fourth, iso, atol=1e-15)


# ---------------------------------------------------------------- moment basis
def test_moment_rows_orthogonal_with_dhumieres_norms():
    G = LAT.M @ LAT.M.T
    off = G - torch.diag(torch.diag(G))
    assert float(off.abs().max()) == 0.0
    assert torch.diag(G).tolist() == GOLD["moment_norms"]["values"]


def test_inverse_is_scaled_transpose():
    norms = torch.tensor(GOLD["moment_norms"]["values"], dtype=torch.float64)
    assert torch.allclose(LAT.Minv, LAT.M.T / norms[None, :], atol=1e-15)


def test_moment_rows_physical_meaning_and_parity():
    M = LAT.M
    assert torch.equal(M[0], torch.ones(19, dtype=torch.float64))
    for k, a in ((3, 0), (5, 1), (7, 2)):
        assert torch.equal(M[k], C[:, a])          # momentum rows
    assert torch.equal(M[13], C[:, 0] * C[:, 1])   # p_xy
    assert torch.equal(M[14], C[:, 1] * C[:, 2])   # p_yz
    assert torch.equal(M[15], C[:, 0] * C[:, 2])   # p_xz
    opp = LAT.opp
    for k in GOLD["moment_parity"]["even"]:
        assert torch.equal(M[k][opp], M[k])
    for k in GOLD["moment_parity"]["odd"]:
        assert torch.equal(M[k][opp], -M[k])


def _feq_incompressible(rho, j):
    """Eq. BGK-EDF with c_s^2 = 1/3 in the incompressible form (rho0 = 1)."""
    cj = C @ j
    jj = (j * j).sum(0)
    return LAT.w[:, None] * (rho[None] + 3 * cj + 4.5 * cj * cj - 1.5 * jj[None])


def test_equilibrium_moments_are_moments_of_bgk_equilibrium():
    g = torch.Generator().manual_seed(0)
    rho = 1 + 0.01 * torch.randn(50, generator=g, dtype=torch.float64)
    j = 0.05 * torch.randn(3, 50, generator=g, dtype=torch.float64)
    meq = O.equilibrium_moments(rho, j)
    assert torch.allclose(LAT.M @ _feq_incompressible(rho, j), meq, atol=1e-14)


def test_guo_source_moments():
    """Guo's source has zero mass, momentum F and second moment uF + Fu."""
    g = torch.Generator().manual_seed(1)
    u = 0.05 * torch.randn(3, 20, generator=g, dtype=torch.float64)
    F = 1e-3 * torch.randn(3, 20, generator=g, dtype=torch.float64)
    Fi = O.guo_source(LAT.c, LAT.w, u, F)
    assert float(Fi.sum(0).abs().max()) < 1e-17
    assert torch.allclose(C.T @ Fi, F, atol=1e-17)
    second = torch.einsum("ia,ib,in->abn", C, C, Fi)
    want = torch.einsum("an,bn->abn", u, F) + torch.einsum("an,bn->abn", F, u)
    assert torch.allclose(second, want, atol=1e-17)


# ---------------------------------------------------------------- rates (Table 2)
def _lam(s):
    return 1.0 / float(s) - 0.5


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 1.3, 2.0])
def test_rate_sets_magic_products(tau):
    lp = tau - 0.5
    sB = O.rates("B", tau)
    assert abs(lp * _lam(sB[4]) - GOLD["set_b_magic"]["Lambda"]) < 1e-14
    assert abs(lp * _lam(sB[16]) - GOLD["set_b_magic"]["Lambda"]) < 1e-14
    sD = O.rates("D", tau)
    assert abs(lp * _lam(sD[4]) - GOLD["set_d_magic"]["Lambda_q"]) < 1e-14
    assert abs(lp * _lam(sD[16]) - GOLD["set_d_magic"]["Lambda_m"]) < 1e-14
    for Lam in (1 / 64, 1 / 12, 3 / 16, 1 / 4, 3 / 8, 1.0):
        sE = O.rates("E", tau, Lam)
        assert abs(lp * _lam(sE[4]) - Lam) < 1e-13
        assert abs(lp * _lam(sE[17]) - Lam) < 1e-13
    sA = O.rates("A", tau)
    assert abs(lp * _lam(sA[4]) - 3 / 16) < 1e-14   # A shares B's odd rates


def _table2(tau_key, rset):
    from fractions import Fraction
    return [float(Fraction(v)) for v in GOLD["table2_rates"]["rates"][tau_key][rset]]


@pytest.mark.parametrize("tau_key", ["0.6", "1.3"])
@pytest.mark.parametrize("rset", ["SRT", "A", "B", "C", "D", "E"])
def test_rates_equal_table2_entries(tau_key, rset):
    """All 19 rates of every set against Table 2 evaluated by hand (exact
    fractions, tests/golden/paper_values.json): pins every entry, Set A's
    even-sector rates s_e, s_eps, s_pi included."""
    lam = float(__import__("fractions").Fraction(GOLD["table2_rates"]["Lambda_E"]))
    got = O.rates(rset, float(tau_key), lam if rset == "E" else None).numpy()
    assert np.allclose(got, _table2(tau_key, rset), rtol=0, atol=1e-15)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.3])
def test_rate_sets_structure(tau):
    s = 1 / tau
    for rs in O.SETS:
        r = O.rates(rs, tau, 0.2)
        assert r[[0, 3, 5, 7]].abs().max() == 0                       # conserved
        assert torch.allclose(r[[9, 11, 13, 14, 15]], torch.full((5,), s, dtype=torch.float64))
        assert r[4] == r[6] == r[8] and r[16] == r[17] == r[18] and r[10] == r[12]
    c = O.rates("C", tau)
    gc = GOLD["set_c_rates"]
    assert [float(c[1]), float(c[2]), float(c[4]), float(c[10]), float(c[16])] == \
        [gc["s_e"], gc["s_eps"], gc["s_q"], gc["s_pi"], gc["s_m"]]
    srt = O.rates("SRT", tau)
    assert torch.allclose(srt[srt != 0], torch.full((15,), s, dtype=torch.float64))
    # Set E at Lambda = 3/16 has the rates of Set B
    assert torch.allclose(O.rates("E", tau, GOLD["set_e_equivalences"]["set_b_Lambda"]),
                          O.rates("B", tau), atol=1e-15)
    # Lambda = 3/8: odd rates 4(2-s)/(4+s)
    e38 = O.rates("E", tau, GOLD["set_e_equivalences"]["lambda_3_8"])
    assert abs(float(e38[4]) - 4 * (2 - s) / (4 + s)) < 1e-14


def test_set_e_quarter_is_srt_at_tau_one():
    e = GOLD["set_e_equivalences"]
    assert torch.allclose(O.rates("E", e["srt_tau"], e["srt_Lambda"]), O.rates("SRT", e["srt_tau"]))


def test_rates_reject_invalid():
    with pytest.raises(ValueError):
        O.rates("E", 0.5, 0.25)
    with pytest.raises(ValueError):
        O.rates("X", 1.0)
    with pytest.raises(ValueError):
        O.rates("E", 1.0, -0.1)
    with pytest.raises(ValueError):
        O.rates("C", 0.45)


def test_unit_conversion_worked_example():
    u = GOLD["unit_conversion"]
    mD = O.unit_darcy(u["k_lu"], u["dx_m"]) * 1e3
    assert abs(mD / u["k_mD"] - 1) < 2e-4


# ---------------------------------------------------------------- collision
def test_mrt_with_equal_rates_is_bgk_guo():
    """All rates 1/tau: the MRT step equals the BGK collision with Guo forcing
    written directly in velocity space (Sec. 2.1.2, last paragraph)."""
    g = torch.Generator().manual_seed(2)
    tau = 0.83
    rho = 1 + 1e-3 * torch.randn(40, generator=g, dtype=torch.float64)
    j0 = 1e-2 * torch.randn(3, 40, generator=g, dtype=torch.float64)
    f = _feq_incompressible(rho, j0) + 1e-4 * torch.randn(19, 40, generator=g, dtype=torch.float64)
    F = 1e-4 * torch.randn(3, 40, generator=g, dtype=torch.float64)
    out = O.collide(f, O.rates("SRT", tau), F, LAT)
    # velocity-space BGK + Guo
    rho_b = f.sum(0)
    j = C.T @ f + F / 2
    u = j
    cu = C @ u
    feq = LAT.w[:, None] * (rho_b[None] + 3 * cu + 4.5 * cu * cu - 1.5 * (u * u).sum(0)[None])
    cF = C @ F
    Fi = LAT.w[:, None] * (3 * (cF - (u * F).sum(0)[None]) + 9 * cu * cF)
    want = f - (f - feq) / tau + (1 - 0.5 / tau) * Fi
    assert float((out - want).abs().max()) < 1e-15


# ---------------------------------------------------------------- brute force step
def _brute_force_srt_step(fh, solid, tau, F):
    """One pull step, BGK/Guo, written with explicit loops over voxels and links."""
    nz, ny, nx = solid.shape
    c = [tuple(int(a) for a in v) for v in LAT.c]
    opp = [int(a) for a in LAT.opp]
    w = [float(a) for a in LAT.w]
    out = np.zeros_like(fh)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if solid[z, y, x]:
            continue
        f = [0.0] * 19
        for i, (cx, cy, cz) in enumerate(c):
            sx, sy, sz = (x - cx) % nx, (y - cy) % ny, (z - cz) % nz
            f[i] = fh[opp[i], z, y, x] if solid[sz, sy, sx] else fh[i, sz, sy, sx]
        rho = sum(f)
        Fx, Fy, Fz = F
        ux = sum(f[i] * c[i][0] for i in range(19)) + Fx / 2
        uy = sum(f[i] * c[i][1] for i in range(19)) + Fy / 2
        uz = sum(f[i] * c[i][2] for i in range(19)) + Fz / 2
        uu = ux * ux + uy * uy + uz * uz
        for i, (cx, cy, cz) in enumerate(c):
            cu = cx * ux + cy * uy + cz * uz
            feq = w[i] * (rho + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
            cF = cx * Fx + cy * Fy + cz * Fz
            Fi = w[i] * (3 * (cF - (ux * Fx + uy * Fy + uz * Fz)) + 9 * cu * cF)
            out[i, z, y, x] = f[i] - (f[i] - feq) / tau + (1 - 0.5 / tau) * Fi
    return out


def test_stream_bounce_back_against_loop_brute_force():
    mask = random_mask((4, 5, 3), 0.35, seed=7)
    g = (2e-3, -1e-3, 5e-4)
    p = O.Problem(mask, 0.9, None, "SRT", g)
    rng = np.random.default_rng(3)
    fh = p.initial() + 1e-3 * torch.from_numpy(rng.standard_normal((19,) + mask.shape)) * p.fluid[None]
    got, _ = p.step(fh)
    want = _brute_force_srt_step(fh.numpy(), mask != 0, 0.9, g)
    assert np.abs(got.numpy() - want).max() < 1e-15


# ---------------------------------------------------------------- conservation
def test_exact_mass_conservation_random_mask():
    mask = random_mask((8, 8, 8), 0.3, seed=11)
    p = O.Problem(mask, 0.7, 3 / 8, "E", (1e-4, 2e-5, 0))
    fh = p.initial()
    m0 = float(fh.sum())
    for _ in range(1000):
        fh, _ = p.step(fh)
    # FP64 rounding of ~19 terms per node per step, 1000 steps: well below 5e-12
    assert abs(float(fh.sum()) / m0 - 1) < 5e-12


def test_open_box_momentum_growth():
    """No walls: every step adds F to every node, so <u>_n = (n - 1/2) g."""
    mask = np.zeros((3, 4, 5), np.uint8)
    g = np.array([1e-5, -2e-5, 3e-6])
    p = O.Problem(mask, 0.8, None, "D", g)
    r = O.run(p, 6)
    for n in range(1, 7):
        # populations are O(0.3): absolute FP64 resolution of the momentum is ~1e-16
        assert np.allclose(r["umean"][n - 1].numpy(), (n - 0.5) * g, rtol=0, atol=2e-15)


# ---------------------------------------------------------------- closed forms
def _slit_k(H, Ly, Leff):
    return H * (H * H - 1 + 8 * Leff) / (12 * Ly)


@pytest.mark.parametrize("rset,tau,Lam", [("E", 1.0, 3 / 16), ("E", 0.8, 1 / 12), ("E", 1.2, 3 / 8),
                                           ("SRT", 0.8, None), ("B", 1.3, None), ("D", 1.0, None)])
def test_slit_exact_profile_linear(rset, tau, Lam):
    """Plane Poiseuille flow between bounce-back walls: parabola plus a
    Lambda-dependent slip, exact at steady state; Lambda = 3/16 puts the
    no-slip wall exactly midway (Sec. 2.2, Set E)."""
    H, Ly = 8, 10
    m = slit(1, Ly, 1, H)
    g = 1e-6
    p = O.Problem(m, tau, Lam, rset, (g, 0, 0), linear=True)
    r = O.run_to_steady(p, 1e-14, 100000)
    assert r["converged"]
    s = p.s
    lp = tau - 0.5
    Leff = lp * ((1 / float(s[4]) - 0.5) + 3 * (1 / float(s[16]) - 0.5)) / 4
    if rset == "E":
        assert abs(Leff - Lam) < 1e-14
    nu = (tau - 0.5) / 3
    fh = r["state"]
    _, u = p.step(fh)
    y = np.arange(H) - (H - 1) / 2
    want = (g / (2 * nu)) * ((H / 2) ** 2 - y ** 2) + (g / nu) * (16 * Leff - 3) / 24
    got = u[0].numpy()
    assert np.abs(got / want - 1).max() < 1e-8
    assert abs(float(r["k"][0]) / _slit_k(H, Ly, Leff) - 1) < 1e-8


def test_slit_full_equilibrium_deviation_scales_with_g():
    """With the quadratic equilibrium kept, the slit deviates from the linear
    solution by a relative amount proportional to g."""
    H, Ly = 8, 10
    m = slit(1, Ly, 1, H)
    dev = []
    for g in (1e-4, 5e-5):
        p = O.Problem(m, 1.0, 3 / 16, "E", (g, 0, 0))
        r = O.run_to_steady(p, 1e-14, 100000)
        dev.append(float(r["k"][0]) / _slit_k(H, Ly, 3 / 16) - 1)
    assert abs(dev[0]) < 1e-3
    assert abs(dev[1] / dev[0] - 0.5) < 0.05 or max(abs(d) for d in dev) < 1e-10


def _duct_coefficient(nterms=200):
    s = sum(math.tanh(n * math.pi / 2) / n ** 5 for n in range(1, 2 * nterms, 2))
    return (1 - 192 / math.pi ** 5 * s) / 12


def test_square_duct_series():
    """Square duct (textbook series): k = 0.0351443 a^4 / A_cell, errors shrinking with a."""
    coef = _duct_coefficient()
    assert abs(coef - 0.0351443) < 1e-7
    errs = []
    for a in (6, 12):
        m = duct(1, a, wall=1)
        p = O.Problem(m, 1.0, 3 / 16, "E", (1e-6, 0, 0), linear=True)
        r = O.run_to_steady(p, 1e-12, 100000)
        k_exact = coef * a ** 4 / m[:, :, 0].size
        errs.append(abs(float(r["k"][0]) / k_exact - 1))
    assert errs[1] < errs[0]
    assert errs[1] < 0.01


def _sangani_acrivos_k(L, a, c):
    sa = GOLD["sangani_acrivos"]
    chi = c ** (1 / 3)
    invK = sum(co * chi ** p for co, p in zip(sa["coeffs"], sa["powers"]))
    return L ** 3 * invK / (6 * math.pi * a)


def test_simple_cubic_sphere_array_sangani_acrivos():
    """Voxelised sphere in a periodic box vs the Hasimoto / Sangani-Acrivos drag
    at the voxel solid fraction and the volume-equivalent radius; a
    staircase sphere of radius 3-4 voxels lands within a few per cent."""
    for n, R in ((12, 3.0), (16, 4.0)):
        cc = (n - 1) / 2
        m = sphere(n, (cc, cc, cc), R)
        c = float(m.mean())
        a = (3 * m.sum() / (4 * math.pi)) ** (1 / 3)
        p = O.Problem(m, 1.0, 3 / 16, "E", (1e-6, 0, 0))
        r = O.run_to_steady(p, 1e-9, 20000)
        assert r["converged"]
        assert abs(float(r["k"][0]) / _sangani_acrivos_k(n, a, c) - 1) < 0.03


def _k_linear(mask, rset, tau, Lam):
    p = O.Problem(mask, tau, Lam, rset, (1e-6, 0, 0), linear=True)
    r = O.run_to_steady(p, 1e-11, 6000)
    assert r["converged"]
    return float(r["k"][0])


def test_tau_independence_sets_b_d_e_not_a_c_srt():
    """Sets B, D, E (fixed Lambda products) give tau-independent k; A, C and
    SRT do not (Sec. 3.1, Sec. 3.3)."""
    from lbm_inputs import percolating_x
    m = percolating_x(random_mask((7, 7, 7), 0.25, seed=5))
    taus = (0.7, 1.3)
    for rs, Lam in (("B", None), ("D", None), ("E", 1 / 12)):
        k = [_k_linear(m, rs, t, Lam) for t in taus]
        assert abs(k[1] / k[0] - 1) < 1e-8, rs
    for rs in ("A", "C", "SRT"):
        k = [_k_linear(m, rs, t, None) for t in taus]
        assert abs(k[1] / k[0] - 1) > 1e-3, rs


# ---------------------------------------------------------------- TRT (Sec. 2.1.2)
def test_velocity_space_equilibrium_has_the_equilibrium_moments():
    g = torch.Generator().manual_seed(11)
    rho = 0.01 * torch.randn(30, generator=g, dtype=torch.float64)
    j = 0.05 * torch.randn(3, 30, generator=g, dtype=torch.float64)
    for linear in (False, True):
        feq = O.equilibrium(LAT.c, LAT.w, rho, j, linear)
        assert torch.allclose(LAT.M @ feq, O.equilibrium_moments(rho, j, linear), atol=1e-15)


@pytest.mark.parametrize("rset,tau,Lam", [("SRT", 0.7, None), ("SRT", 1.4, None), ("B", 0.8, None),
                                           ("B", 1.6, None), ("E", 1.0, 3 / 16), ("E", 0.6, 1 / 64),
                                           ("E", 1.3, 3 / 8)])
@pytest.mark.parametrize("linear", [False, True])
def test_trt_collision_equals_mrt_for_two_rate_sets(rset, tau, Lam, linear):
    """The link-wise two-rate collision in velocity space and the moment-space
    MRT collision are one map for SRT, B and E: checked on random states and
    forces, including the momentum gain F."""
    g = torch.Generator().manual_seed(12)
    f = LAT.w[:, None] * (1 + 0.02 * torch.randn(19, 64, generator=g, dtype=torch.float64))
    F = 1e-3 * torch.randn(3, 64, generator=g, dtype=torch.float64)
    s = O.rates(rset, tau, Lam)
    a = O.collide(f, s, F, LAT, linear)
    b = O.collide_trt(f, s, F, LAT, linear)
    assert float((a - b).abs().max()) < 1e-15
    assert torch.allclose(C.T @ b, C.T @ f + F, atol=1e-16)


@pytest.mark.parametrize("rset", ["A", "C", "D"])
def test_trt_rejects_sets_that_are_not_two_rate(rset):
    with pytest.raises(ValueError):
        O.trt_rates(O.rates(rset, 0.9, None))
    with pytest.raises(ValueError):
        O.Problem(np.zeros((3, 3, 3), np.uint8), 0.9, None, rset, (1e-6, 0, 0), collision="trt")


def test_trt_slit_exact_profile():
    """TRT alone reproduces the slit's exact steady profile at Lambda_eff (Set E)."""
    H, Ly, tau, Lam, g = 8, 10, 0.8, 1 / 12, 1e-6
    p = O.Problem(slit(1, Ly, 1, H), tau, Lam, "E", (g, 0, 0), linear=True, collision="trt")
    r = O.run_to_steady(p, 1e-14, 100000)
    assert r["converged"]
    nu = (tau - 0.5) / 3
    _, u = p.step(r["state"])
    y = np.arange(H) - (H - 1) / 2
    want = (g / (2 * nu)) * ((H / 2) ** 2 - y ** 2) + (g / nu) * (16 * Lam - 3) / 24
    assert np.abs(u[0].numpy() / want - 1).max() < 1e-8


# ---------------------------------------------------------------- symmetry planes, full-way bounce-back (Sec. 2.3)
def _mirror_yz(m):
    mm = np.concatenate([m, m[:, ::-1, :]], axis=1)
    return np.concatenate([mm, mm[::-1]], axis=0)


def test_symmetry_planes_equal_the_mirrored_periodic_box():
    """Mirror planes on the y and z faces are the periodic box of the image
    reflected in y and z, restricted to the original quarter."""
    m = random_mask((5, 6, 7), 0.3, 3)
    ps = O.Problem(m, 0.9, 3 / 16, "E", (1e-4, 0, 0), symmetric="yz")
    pm = O.Problem(_mirror_yz(m), 0.9, 3 / 16, "E", (1e-4, 0, 0))
    a, b = ps.initial(), pm.initial()
    nz, ny, _ = m.shape
    for _ in range(30):
        a, ua = ps.step(a)
        b, ub = pm.step(b)
    assert float((a - b[:, :nz, :ny, :]).abs().max()) < 1e-14
    # the driven component; transverse means cancel over the mirrored box only
    assert abs(float(ps.mean_velocity(ua)[0] / pm.mean_velocity(ub)[0]) - 1) < 1e-12


def test_symmetry_plane_closes_a_half_slit():
    """A wall below and a mirror plane above: half of the slit of twice the
    height, with its exact profile (Set E, linear equilibrium)."""
    H, tau, Lam, g = 5, 0.8, 1 / 12, 1e-6
    m = np.zeros((1, H + 1, 1), np.uint8)
    m[:, 0, :] = 1
    p = O.Problem(m, tau, Lam, "E", (g, 0, 0), linear=True, symmetric="y")
    r = O.run_to_steady(p, 1e-14, 100000)
    assert r["converged"]
    _, u = p.step(r["state"])
    nu = (tau - 0.5) / 3
    y = np.arange(1, H + 1) - (H + 0.5)
    want = (g / (2 * nu)) * (H * H - y ** 2) + (g / nu) * (16 * Lam - 3) / 24
    assert np.abs(u[0].numpy() / want - 1).max() < 1e-8


def test_symmetry_planes_open_box_accelerates_freely():
    p = O.Problem(np.zeros((4, 5, 3), np.uint8), 1.0, 3 / 16, "E", (1e-5, 0, 0), symmetric="yz")
    r = O.run(p, 20)
    n = np.arange(1, 21)
    assert np.abs(r["umean"][:, 0].numpy() - (n - 0.5) * 1e-5).max() < 2e-15
    assert float(r["umean"][:, 1:].abs().max()) < 1e-15


def test_fullway_bounce_back_reads_the_older_state_at_walls():
    """Full-way bounce-back: at a wall link the population comes back from the
    state one step older; every other link pulls as before."""
    lat = O.Lattice.make()
    m = random_mask((4, 5, 6), 0.35, 9)
    solid = torch.from_numpy(m != 0)
    g = torch.Generator().manual_seed(4)
    fh = torch.randn((19,) + m.shape, generator=g, dtype=torch.float64)
    old = torch.randn((19,) + m.shape, generator=g, dtype=torch.float64)
    half = O.stream(fh, solid, lat)
    full = O.stream_general(fh, solid, lat, fh_wall=old)
    for i in range(19):
        cx, cy, cz = (int(v) for v in lat.c[i])
        wall = torch.roll(solid, shifts=(cz, cy, cx), dims=(0, 1, 2))
        assert torch.equal(full[i][~wall], half[i][~wall])
        assert torch.equal(full[i][wall], old[int(lat.opp[i])][wall])


def test_fullway_steady_state_equals_halfway():
    """Full-way bounce-back only delays wall reflections by one step, so the
    steady state at fluid nodes is the halfway one (linear equilibrium)."""
    m = percolating_x(random_mask((7, 7, 7), 0.25, 5))
    ks = []
    for fw in (False, True):
        p = O.Problem(m, 1.0, 3 / 16, "E", (1e-5, 0, 0), linear=True, fullway=fw)
        r = O.run_to_steady(p, 1e-13, 200000)
        assert r["converged"]
        ks.append(float(r["k"][0]))
    assert abs(ks[1] / ks[0] - 1) < 1e-9


# ---------------------------------------------------------------- Zou-He pressure boundaries (Sec. 2.3, 3.1)
def test_zou_he_sets_density_and_zero_transverse_velocity():
    lat = O.Lattice.make()
    g = torch.Generator().manual_seed(6)
    f = lat.w[:, None, None, None] * (1 + 0.01 * torch.randn((19, 3, 4, 5), generator=g, dtype=torch.float64))
    rin, rout = 1.0003, 0.9996
    f = O.zou_he_pressure(f, lat, rin, rout)
    c = lat.c.to(torch.float64)
    for plane, rho in ((0, rin), (4, rout)):
        fp = f[..., plane]
        assert torch.allclose(fp.sum(0), torch.full_like(fp.sum(0), rho), atol=1e-15)
        for a in (1, 2):
            assert float((c[:, a][:, None, None] * fp).sum(0).abs().max()) < 1e-16
        # non-equilibrium bounce-back along x: f1 - f1eq = f2 - f2eq at (rho, (u_x, 0, 0))
        ux = (c[:, 0][:, None, None] * fp).sum(0) / 1.0
        j = torch.stack([ux, torch.zeros_like(ux), torch.zeros_like(ux)]).reshape(3, -1)
        feq = O.equilibrium(lat.c, lat.w, torch.full_like(ux, rho).reshape(-1), j, linear=True)
        neq = fp.reshape(19, -1) - feq
        i = int(torch.nonzero((lat.c == torch.tensor([1, 0, 0])).all(1))[0])
        assert float((neq[i] - neq[int(lat.opp[i])]).abs().max()) < 1e-15


@pytest.mark.parametrize("nx", [12])
def test_pressure_driven_slit_exact_at_lambda_quarter(nx):
    """Zou-He inlet/outlet and halfway walls: at Lambda = 1/4 the pressure-driven
    slit has the closed-form permeability, k from the pressure drop over nx - 1
    (Eq. perm_calc)."""
    H, Ly = 8, 10
    p = O.Problem(slit(nx, Ly, 1, H), 0.8, 1 / 4, "E", (0, 0, 0), linear=True, pressure=(1 + 5e-5, 1 - 5e-5))
    r = O.run_to_steady(p, 1e-13, 400000)
    assert r["converged"]
    assert abs(float(r["k"][0]) / _slit_k(H, Ly, 1 / 4) - 1) < 1e-9


def test_pressure_driven_slit_error_falls_with_length():
    """Away from Lambda = 1/4 the boundary planes leave an O(1/nx) error in k."""
    H, Ly = 8, 10
    err = []
    for nx in (12, 24):
        p = O.Problem(slit(nx, Ly, 1, H), 0.8, 1 / 12, "E", (0, 0, 0), linear=True, pressure=(1 + 5e-5, 1 - 5e-5))
        r = O.run_to_steady(p, 1e-13, 400000)
        err.append(abs(float(r["k"][0]) / _slit_k(H, Ly, 1 / 12) - 1))
    assert err[0] < 2e-3
    assert abs(err[1] / err[0] - 0.5) < 0.05
