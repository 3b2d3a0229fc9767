"""FP16 storage with a per-node reference density (LBM_F16R): layout and
host round trips, table/bitmap agreement, and the step against the oracle
from a random state.  The stored values are velocity-sized, so one step
keeps the populations to FP16 rounding of that part (2^-11 relative) rather
than of the density deviation."""
import numpy as np
import pytest

import oracle as O
import paper_1902_11193_amd as P
from gpu_helpers import banner, dense_from_lib, lib_from_dense, random_state, deviation_error, W_LIB
from lbm_inputs import random_mask

pytestmark = pytest.mark.gpu


def _state_with_density(nf, seed):
    """A random state whose density deviation is 1e3 times its velocity part,
    as in poorly connected rock."""
    rng = np.random.default_rng(seed)
    drho = 1e-3 * rng.standard_normal(nf)
    f = W_LIB[:, None] * (1.0 + drho[None, :])
    return f + 1e-6 * rng.standard_normal((19, nf))


def test_f16r_state_roundtrip_keeps_the_small_part():
    mask = random_mask((8, 9, 10), 0.3, 4)
    banner("f16r roundtrip")
    res = {}
    for storage in ("f16", "f16r"):
        s = P.Solver(mask, 1.0, 3 / 16, "E", (1e-6, 0, 0), storage)
        f0 = _state_with_density(s.n_fluid, 1)
        s.set_state(f0)
        f1 = s.get_state()
        # error relative to the velocity-sized part f - w (1 + drho)
        rho = f0.sum(0)
        small = f0 - W_LIB[:, None] * rho[None, :]
        res[storage] = np.abs(f1 - f0).max() / np.abs(small).max()
        s.close()
    assert res["f16r"] < 2e-3, res          # FP16 rounding of the small part (+ reference rounding)
    assert res["f16"] > 10 * res["f16r"], res


@pytest.mark.parametrize("shape", [(9, 10, 70), (300, 4, 5)])   # one z-tile; three 128-plane tiles
def test_f16r_table_and_bitmap_bitwise_equal(shape):
    mask = random_mask(shape, 0.3, 5)
    banner(f"f16r table vs bitmap {shape}")
    out = []
    for index in ("table", "bitmap"):
        s = P.Solver(mask, 0.9, 1 / 12, "E", (1e-5, 0, 0), "f16r", index)
        s.set_state(_state_with_density(s.n_fluid, 2))
        s.step(20)
        out.append((s.get_state(), s.history(20)))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("shape", [(8, 8, 8), (300, 3, 4)])     # one z-tile; three 128-plane tiles
@pytest.mark.parametrize("index", ["table", "bitmap"])
def test_f16r_steps_match_oracle(index, shape):
    """From a density-dominated random state, 1, 2 and 20 steps against the
    FP64 oracle, errors measured on the velocity-sized part."""
    mask = random_mask(shape, 0.3, 11)
    banner(f"f16r vs oracle {index} {shape}")
    s = P.Solver(mask, 0.9, 3 / 16, "E", (1e-5, 0, 0), "f16r", index)
    s.set_state(_state_with_density(s.n_fluid, 3))
    f0 = s.get_state()
    p = O.Problem(mask, 0.9, 3 / 16, "E", (1e-5, 0, 0))
    fh = dense_from_lib(p, f0)
    done = 0
    for n in (1, 2, 20):
        s.step(n - done)
        for _ in range(n - done):
            fh, u = p.step(fh)
        done = n
        ref = lib_from_dense(p, fh)
        small = ref - W_LIB[:, None] * ref.sum(0)[None, :]
        err = np.abs(s.get_state() - ref).max() / np.abs(small).max()
        assert err < 5e-3, (index, n, err)
    s.close()


def test_f16r_exponent_change_keeps_the_reference():
    mask = random_mask((8, 8, 8), 0.3, 1)
    banner("f16r exponent")
    s = P.Solver(mask, 1.0, 3 / 16, "E", (1e-4, 0, 0), "f16r")
    s.set_state(_state_with_density(s.n_fluid, 6))
    s.step(5)
    f1 = s.get_state()
    s.set_storage_exponent(12)
    f2 = s.get_state()
    small = f1 - W_LIB[:, None] * f1.sum(0)[None, :]
    assert np.abs(f1 - f2).max() < 2e-3 * np.abs(small).max()
    s.close()
