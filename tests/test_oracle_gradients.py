"""Pins for the oracle's discrete adjoint (reverse-mode through the FP64 forward).

Checked against central finite differences of the forward in FP64, against
the exact Euler identity of the linearised scheme, and against the slit's
closed-form derivatives of k(tau, Lambda).
"""
import numpy as np
import pytest

import oracle as O
from lbm_inputs import slit, random_mask, percolating_x

MASK = percolating_x(random_mask((5, 6, 7), 0.25, seed=21))


def _k(mask, tau, Lam, rset, g_field, n, linear=False, gref=1e-5):
    p = O.Problem(mask, tau, Lam, rset, (gref, 0, 0), g_field=g_field, linear=linear)
    return float(O.run(p, n, keep_state=False)["k"][0])


def _uniform(mask, gx):
    g = np.zeros((3,) + mask.shape)
    g[0] = gx
    return g


@pytest.mark.parametrize("rset,Lam", [("E", 3 / 16), ("SRT", None), ("D", None)])
def test_gradients_match_central_differences(rset, Lam):
    n, tau, gref = 40, 0.9, 1e-5
    p = O.Problem(MASK, tau, Lam, rset, (gref, 0, 0))
    gr = O.gradients(p, n, segment=7)
    gf = _uniform(MASK, gref)
    h = 1e-4
    fd_tau = (_k(MASK, tau + h, Lam, rset, gf, n) - _k(MASK, tau - h, Lam, rset, gf, n)) / (2 * h)
    scale = max(abs(fd_tau), gr["k"] / tau)
    assert abs(gr["dk_dtau"] - fd_tau) < 1e-6 * scale
    if rset == "E":
        fd_l = (_k(MASK, tau, Lam + h, rset, gf, n) - _k(MASK, tau, Lam - h, rset, gf, n)) / (2 * h)
        assert abs(gr["dk_dLambda"] - fd_l) < 1e-6 * max(abs(fd_l), gr["k"])
    else:
        assert gr["dk_dLambda"] == 0.0
    fluid = np.flatnonzero(MASK.reshape(-1) == 0)
    rng = np.random.default_rng(0)
    for idx in rng.choice(len(fluid), 4, replace=False):
        for comp in (0, 1):
            vox = np.unravel_index(fluid[idx], MASK.shape)
            dg = h * gref
            gp, gm = gf.copy(), gf.copy()
            gp[(comp,) + vox] += dg
            gm[(comp,) + vox] -= dg
            fd = (_k(MASK, tau, Lam, rset, gp, n) - _k(MASK, tau, Lam, rset, gm, n)) / (2 * dg)
            ad = float(gr["dk_dg"][comp, idx])
            assert abs(ad - fd) < 1e-6 * max(abs(fd), gr["k"] / gref / len(fluid))


def test_euler_identity_linear_scheme():
    """The linearised scheme is linear in g, so sum_x g0 dk/dg_x(x) = k exactly."""
    gref = 1e-5
    p = O.Problem(MASK, 1.1, 1 / 12, "E", (gref, 0, 0), linear=True)
    gr = O.gradients(p, 60, segment=16)
    s = float(gr["dk_dg"][0].sum()) * gref
    assert abs(s / gr["k"] - 1) < 1e-10


@pytest.mark.parametrize("rset,tau,Lam", [("E", 1.0, 3 / 16), ("SRT", 0.9, None)])
def test_slit_closed_form_gradients(rset, tau, Lam):
    """Slit: k = H (H^2 - 1 + 8 Lambda_eff) / (12 L_y), Lambda_eff = Lambda (Set E)
    or (tau - 1/2)^2 (SRT): dk/dLambda = 2H/(3 L_y), dk/dtau = 0 for Set E;
    dk/dtau = 4 H (tau - 1/2) / (3 L_y) for SRT."""
    H, Ly = 8, 10
    m = slit(1, Ly, 1, H)
    p = O.Problem(m, tau, Lam, rset, (1e-6, 0, 0), linear=True)
    gr = O.gradients(p, 2500, segment=250)
    if rset == "E":
        assert abs(gr["dk_dLambda"] / (2 * H / (3 * Ly)) - 1) < 1e-6
        assert abs(gr["dk_dtau"]) < 1e-6 * gr["k"]
    else:
        assert abs(gr["dk_dtau"] / (4 * H * (tau - 0.5) / (3 * Ly)) - 1) < 1e-6


def test_stored_oracle_gradient_at_full_size_settings_agrees_with_finite_differences():
    """tests/golden/pack_crop32_adjoint.json (written by make_golden.py from the
    oracle alone): at the adjoint's full-size settings, 4000 steps with
    segments of 200 on a 32^3 pack crop, the oracle's reverse-mode gradient
    matches FP64 central differences of its own k -- h = 1e-4 in tau and
    Lambda, a 1e-2 relative change of g_x at four single voxels -- to 1e-4."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pack_crop32_adjoint.json")))
    k = gold["k"]
    assert abs(gold["dk_dtau"] - gold["fd_dk_dtau"]) < 1e-4 * max(abs(gold["fd_dk_dtau"]), k)
    assert abs(gold["dk_dLambda"] / gold["fd_dk_dLambda"] - 1) < 1e-4
    for node, fd in gold["fd_dk_dgx"].items():
        adj = gold["dk_dgx_sample"][gold["sample"].index(int(node))]
        assert abs(adj / fd - 1) < 1e-4, (node, adj, fd)
    # Euler identity for the nearly linear scheme: sum g0 dk/dg = k
    assert abs(gold["dk_dgx_sum"] * 1e-6 / k - 1) < 1e-4
