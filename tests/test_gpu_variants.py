"""Every step-kernel variant the library launches on the bitmap index --
storage FP32 / FP16 / BF16 / F16R, moment-space or link-wise collision,
uniform or per-node body force -- takes one step from a random state as the
FP64 oracle does from the same (decoded) state.

Set E is a two-rate set, so the link-wise TRT kernel computes the oracle's
moment-space collision as well.  Bounds: FP32 rounding (2e-6 of the
deviation scale); for the half types, half an ulp of the stored value
(2^-11 / 2^-8 relative, checked at twice that); for F16R, FP16 rounding of the
part left after the reference density."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1902_11193_amd as P
from gpu_helpers import banner, dense_from_lib, lib_from_dense, random_state, deviation_error, W_LIB
from lbm_inputs import random_mask

pytestmark = pytest.mark.gpu

G = (1e-4, 3e-5, -2e-5)
TAU, LAM = 0.9, 3 / 16


@pytest.mark.parametrize("field", [False, True], ids=["uniform", "field"])
@pytest.mark.parametrize("collision", ["mrt", "trt"])
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "f16r"])
def test_one_step_of_every_variant(storage, collision, field):
    mask = random_mask((7, 9, 23), 0.3, 31)
    banner(f"variant {storage} {collision} {'field' if field else 'uniform'}")
    s = P.Solver(mask, TAU, LAM, "E", G, storage, "bitmap")
    s.set_collision(collision)
    nf = s.n_fluid
    s.set_state(random_state(nf, 17))
    f0 = s.get_state()                       # the start as the GPU holds it
    g_dense = None
    if field:
        rng = np.random.default_rng(8)
        gf = (np.array(G)[:, None] * (1 + 0.5 * rng.standard_normal((3, nf)))).astype(np.float32)
        s.set_force_field(torch.from_numpy(gf).cuda())
        g_dense = np.zeros((3,) + mask.shape)
        g_dense.reshape(3, -1)[:, P.lbm_node_order(mask)] = gf.astype(np.float64)
    p = O.Problem(mask, TAU, LAM, "E", G, g_field=g_dense)
    fh, _ = p.step(dense_from_lib(p, f0))
    want = lib_from_dense(p, fh)
    s.step(1)
    got = s.get_state()
    s.close()
    if storage == "f32":
        assert deviation_error(got, want) < 2e-6
    elif storage == "f16r":
        small = want - W_LIB[:, None] * want.sum(0)[None, :]
        assert np.abs(got - want).max() < 2e-3 * np.abs(small).max()
    else:
        assert deviation_error(got, want) < (2.0**-10 if storage == "f16" else 2.0**-7)
