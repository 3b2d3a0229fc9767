"""Captured-graph replay of 32-step stretches (lbm_set_graphs): every replay
must give the same state and per-step history as plain launches, bit for
bit, including across settings changes that drop the graphs.  The replays
are interleaved with the program's own eager work and host synchronisation
(state reads, single steps)."""
import numpy as np
import pytest

import paper_1902_11193_amd as P
from gpu_helpers import banner, random_state
from lbm_inputs import random_mask, pipe

pytestmark = pytest.mark.gpu

G = (1e-5, 2e-6, 0.0)


def _pair(mask, storage="f32", rset="E", tau=0.9, Lam=3 / 16):
    a = P.Solver(mask, tau, Lam, rset, G, storage, "bitmap")
    b = P.Solver(mask, tau, Lam, rset, G, storage, "bitmap")
    b.set_graphs(False)
    f0 = random_state(a.n_fluid, 4)
    a.set_state(f0)
    b.set_state(f0)
    return a, b


@pytest.mark.parametrize("storage", ["f32", "f16r"])
def test_graph_replays_equal_plain_launches(storage):
    mask = random_mask((9, 10, 11), 0.3, 8)
    banner(f"graphs vs plain {storage}")
    a, b = _pair(mask, storage)
    for n in (1, 32, 65, 31, 96, 3):          # replays start once a step is pending
        a.step(n)
        b.step(n)
        assert np.array_equal(a.get_state(), b.get_state()), n
        h = min(a.steps_done, 1000)
        assert np.array_equal(a.history(h), b.history(h)), n
    a.close()
    b.close()


def test_graphs_follow_settings_changes():
    mask = random_mask((8, 8, 12), 0.3, 9)
    banner("graphs across settings")
    a, b = _pair(mask, "f32", "E", 1.0, 3 / 16)
    for s in (a, b):
        s.step(40)
        s.set_collision("trt")
        s.step(70)
        s.set_collision("mrt")
        s.set_storage_exponent(0)
        s.step(64)
    assert np.array_equal(a.get_state(), b.get_state())
    assert np.array_equal(a.history(174), b.history(174))
    a.close()
    b.close()


def test_run_to_steady_with_graphs():
    mask = pipe(4, 24, 8.0)
    banner("run_to_steady graphs")
    res = []
    for graphs in (True, False):
        s = P.Solver(mask, 0.8, 3 / 16, "E", (1e-6, 0, 0))
        s.set_graphs(graphs)
        res.append(s.run_to_steady(eps=1e-9, check_every=100, max_steps=20000))
        s.close()
    assert res[0]["steps"] == res[1]["steps"] and res[0]["converged"] == res[1]["converged"]
    assert np.array_equal(res[0]["k"], res[1]["k"], equal_nan=True)   # k_y, k_z are NaN (no force)
