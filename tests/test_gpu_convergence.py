"""GPU parity of the stopping rule (Eq. convergence, Sec. 3) and of the
permeability of the 32^3 simple-cubic sphere array (BASELINE's first
configuration) against the Sangani-Acrivos drag.

lbm_run_to_steady checks the per-step relative change of k every
`check_every` steps from the device history; it must stop in the chunk that
holds the step where the FP64 oracle's oracle.run_to_steady stops, and k
at that step must agree to 1e-6.  Near the threshold FP32 storage moves the
per-step change by ~1e-8 relative to k, so the first step under eps may
shift by a step or two; the check allows two.  The same noise sets a floor
on the criterion itself: with FP32 storage a per-step change below ~1e-8
is rounding, not flow, and a test at eps = 1e-9 can hold early (on the slit
below at step 2903 against the oracle's 3933), so the tests use the paper's
eps = 1e-6."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import paper_1902_11193_amd as P
from gpu_helpers import banner
from lbm_inputs import pipe, slit, workload

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CHECK = 100


def first_hit(u, first_step, eps):
    """First step n (numbered from first_step for u[0]) with
    |u_n - u_(n-1)| < eps |u_n|, n >= 2; None if none."""
    rel = np.abs(np.diff(u)) / np.abs(u[1:])
    for j in np.flatnonzero(rel < eps):
        n = first_step + 1 + int(j)
        if n >= 2:
            return n
    return None


def gpu_stop(s, eps, max_steps):
    r = s.run_to_steady(eps=eps, check_every=CHECK, max_steps=max_steps)
    done = r["steps"]
    m = min(done, 2 * CHECK + 1)
    u = s.history(m)[:, 0]
    return r, first_hit(u, done - m + 1, eps), dict(zip(range(done - m + 1, done + 1), u))


@pytest.mark.parametrize("name,make,tau,rset,Lam", [
    ("slit H=16", lambda: slit(4, 18, 4, 16), 0.8, "E", 3 / 16),
    ("slit H=12 SRT", lambda: slit(4, 14, 4, 12), 1.3, "SRT", None),
    ("pipe D=16", lambda: pipe(4, 20, 8.0), 1.2, "D", None),
    ("pipe D=12 A", lambda: pipe(4, 16, 6.0), 0.7, "A", None),
])
def test_run_to_steady_stops_where_the_oracle_stops(name, make, tau, rset, Lam):
    eps = 1e-6
    mask = make()
    g = (1e-5, 0.0, 0.0)
    banner(f"run_to_steady {name} eps={eps}")
    p = O.Problem(mask, tau, Lam, rset, g)
    ro = O.run_to_steady(p, eps, 20000)
    assert ro["converged"]
    n_o, k_o = ro["steps"], float(ro["k"][0])
    s = P.Solver(mask, tau, Lam, rset, g)
    r, n_g, hist = gpu_stop(s, eps, 20000)
    print(f"{name} eps={eps}: oracle stops at {n_o}, GPU test first holds at {n_g}, GPU returned after {r['steps']}")
    assert r["converged"] and n_g is not None
    assert abs(n_g - n_o) <= 2
    assert r["steps"] == math.ceil(n_g / CHECK) * CHECK
    nu = (tau - 0.5) / 3.0
    k_g = nu * hist[n_o] / g[0]
    assert abs(k_g / k_o - 1) < 1e-6, (k_g, k_o)
    s.close()


def test_run_to_steady_sphere_array_paper_criterion():
    """The 32^3 sphere array (R = 8, tau = 1, Set E, Lambda = 3/16) with the
    paper's eps = 1e-6: the oracle stops at the step stored in
    tests/golden/sc_sphere_32_steady.json."""
    gold = json.load(open(os.path.join(GOLD, "sc_sphere_32_steady.json")))
    banner("run_to_steady sc_sphere_32 eps=1e-6")
    s = P.Solver(workload("sc_sphere_32"), 1.0, 3 / 16, "E", (1e-6, 0, 0))
    r, n_g, hist = gpu_stop(s, gold["eps"], gold["max_steps"])
    print(f"sc_sphere_32: oracle stops at {gold['steps']}, GPU test first holds at {n_g}, returned after {r['steps']}")
    assert gold["converged"] and r["converged"]
    assert abs(n_g - gold["steps"]) <= 2
    assert r["steps"] == math.ceil(n_g / CHECK) * CHECK
    k_g = (0.5 / 3.0) * hist[gold["steps"]] / 1e-6
    assert abs(k_g / gold["k_x"] - 1) < 1e-6
    s.close()


def sangani_acrivos_k(L, n_solid):
    """k of a simple-cubic array of spheres of the voxel solid fraction,
    Hasimoto / Sangani-Acrivos series (coefficients in paper_values.json):
    force per sphere = rho0 g L^3 = 6 pi mu a U K, k = nu <u> / g = L^3 / (6 pi a K),
    a the volume-equivalent radius."""
    sa = json.load(open(os.path.join(GOLD, "paper_values.json")))["sangani_acrivos"]
    c = n_solid / L ** 3
    chi = c ** (1.0 / 3.0)
    inv_K = sum(a * chi ** p for a, p in zip(sa["coeffs"], sa["powers"]))
    a = (3.0 * n_solid / (4.0 * math.pi)) ** (1.0 / 3.0)
    return L ** 3 * inv_K / (6.0 * math.pi * a)


def test_sphere_array_permeability_vs_sangani_acrivos():
    """The same array stepped until the two-step mean of k changes by less
    than 1e-10 per step: k within 3% of the Sangani-Acrivos value for the
    voxelised sphere (volume-equivalent radius; the staircase surface and
    halfway bounce-back place the wall to within a fraction of a voxel)."""
    m = workload("sc_sphere_32")
    banner("sc_sphere_32 vs Sangani-Acrivos")
    s = P.Solver(m, 1.0, 3 / 16, "E", (1e-6, 0, 0))
    prev = None
    for _ in range(200):
        s.step(500)
        u = s.history(2)[:, 0].mean()
        if prev is not None and abs(u - prev) < 1e-10 * 500 * abs(u):
            break
        prev = u
    k = (0.5 / 3.0) * u / 1e-6
    k_sa = sangani_acrivos_k(32, int(m.sum()))
    print(f"sc_sphere_32: k = {k:.6f} after {s.steps_done} steps, Sangani-Acrivos {k_sa:.6f}, "
          f"rel {k / k_sa - 1:+.4%}")
    assert abs(k / k_sa - 1) < 0.03
    s.close()
