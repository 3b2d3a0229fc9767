"""GPU parity of the link-wise TRT collision kernel (Sec. 2.1.2) for the
two-rate sets SRT, B and E: populations against the oracle's velocity-space
TRT collision and against the library's own moment-space MRT kernel, at the
same bound as the MRT parity tests (2e-6 of the deviation scale after 1, 2 and
50 steps from a random state)."""
import numpy as np
import pytest

import oracle as O
import paper_1902_11193_amd as P
from gpu_helpers import banner, dense_from_lib, lib_from_dense, random_state, deviation_error
from lbm_inputs import random_mask, sphere, percolating_x

pytestmark = pytest.mark.gpu

G = (1e-4, 5e-5, -2e-5)
CASES = [
    ("rand8", lambda: random_mask((8, 8, 8), 0.3, 11)),
    ("rand_ragged", lambda: random_mask((7, 9, 11), 0.35, 12)),
    ("sphere16", lambda: sphere(16, (7.5, 7.5, 7.5), 4.0)),
]
SETS = (("E", 0.8, 3 / 16), ("E", 1.3, 1 / 12), ("SRT", 1.1, None), ("B", 0.6, None))


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("index", ["table", "bitmap"])
def test_trt_populations_match_oracle_and_mrt(name, make, index):
    mask = make()
    for rset, tau, Lam in SETS:
        banner(f"trt {name} {index} {rset} tau={tau}")
        states = {}
        for kind in ("trt", "mrt"):
            s = P.Solver(mask, tau, Lam, rset, G, "f32", index)
            s.set_collision(kind)
            f0 = random_state(s.n_fluid, 7)
            s.set_state(f0)
            f0 = s.get_state()
            got = {}
            for n in (1, 2, 50):
                s.step(n - (0 if not got else max(got)))
                got[n] = (s.get_state(), s.mean_velocity())
            states[kind] = (f0, got)
            s.close()
        f0, got = states["trt"]
        p = O.Problem(mask, tau, Lam, rset, G, collision="trt")
        fh = dense_from_lib(p, f0)
        done = 0
        for n in (1, 2, 50):
            for _ in range(n - done):
                fh, u = p.step(fh)
            done = n
            ref = lib_from_dense(p, fh)
            err = deviation_error(got[n][0], ref)
            assert err < 2e-6, (name, index, rset, n, err)
            uo = p.mean_velocity(u).numpy()
            assert np.allclose(got[n][1], uo, rtol=0, atol=1e-6 * np.abs(uo).max())
            err_mrt = deviation_error(got[n][0], states["mrt"][1][n][0])
            assert err_mrt < 2e-6, (name, index, rset, n, err_mrt)


def test_trt_steady_k_matches_mrt():
    mask = percolating_x(random_mask((7, 7, 7), 0.25, 5))
    banner("trt steady k 7^3")
    ks = {}
    for kind in ("mrt", "trt"):
        s = P.Solver(mask, 0.9, 3 / 16, "E", (1e-5, 0, 0), "f32", "bitmap")
        s.set_collision(kind)
        s.step(3000)
        ks[kind] = float(s.permeability()[0])
        s.close()
    assert abs(ks["trt"] / ks["mrt"] - 1) < 1e-5, ks


@pytest.mark.parametrize("rset", ["A", "C", "D"])
def test_set_collision_rejects_sets_that_are_not_two_rate(rset):
    mask = random_mask((6, 6, 6), 0.3, 2)
    banner(f"set_collision reject {rset}")
    s = P.Solver(mask, 0.9, None, rset, G, "f32", "bitmap")
    with pytest.raises(P.LbmError) as e:
        s.set_collision("trt")
    assert e.value.code == P.LBM_EINVAL
    s.step(3)                       # the context still steps with MRT
    assert np.isfinite(s.mean_velocity()).all()
    s.close()
