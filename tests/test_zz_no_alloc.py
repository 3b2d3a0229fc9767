"""lbm_setup_static (the reduction scratch in the library's static array, for
callers that cannot allocate) against lbm_setup: two setups in a row, the
second on a smaller image, each stepped and compared bit for bit with a
context set up with lbm_setup on the same image (same kernels, same launch
shape, the same fixed-order reductions).  While a static context is alive a
second one on the same GPU is refused with LBM_EBUSY."""
import numpy as np
import pytest

import paper_1902_11193_amd as P
from gpu_helpers import banner, random_state
from lbm_inputs import percolating_x, random_mask

pytestmark = pytest.mark.gpu

G = (1e-5, 2e-6, -1e-6)


def _run(mask, static, storage):
    s = P.Solver(mask, 0.9, 3 / 16, "E", G, storage, "bitmap", static_scratch=static)
    s.set_state(random_state(s.n_fluid, 4))
    s.step(70)                                   # past two replayed 32-step graphs
    out = dict(state=s.get_state(), hist=s.history(70), k=s.permeability(), dm=s.mass_deviation())
    r = s.run_to_steady(eps=1e-6, check_every=50, max_steps=300)
    out.update(steady=(r["steps"], r["converged"], r["k"]), hist2=s.history(50))
    return s, out


def test_static_scratch_setup_matches_lbm_setup():
    cases = [((22, 26, 30), 0.3, 1, "f32"), ((9, 11, 13), 0.35, 2, "f16r")]   # the second smaller
    for call, (shape, solid, seed, storage) in enumerate(cases):
        mask = percolating_x(random_mask(shape, solid, seed))
        banner(f"static scratch call {call}: {shape} {storage}")
        ref, want = _run(mask, False, storage)
        ref.close()
        s, got = _run(mask, True, storage)
        for key in ("state", "hist", "k", "hist2"):
            assert np.array_equal(got[key], want[key], equal_nan=True), (call, key)
        assert got["dm"] == want["dm"] and got["steady"][:2] == want["steady"][:2]
        assert np.array_equal(got["steady"][2], want["steady"][2], equal_nan=True)
        with pytest.raises(P.LbmError) as e:
            P.Solver(mask, 0.9, 3 / 16, "E", G, storage, "bitmap", static_scratch=True)
        assert e.value.code == P.LBM_EBUSY
        s.close()
