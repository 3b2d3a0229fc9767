"""Half-precision storage codecs of the step: the value a step stores in FP16
(x 2^e) or BF16 is the FP32 result rounded to nearest, ties to even.

Both storages run the same FP32 collision; started from a state whose
deviations are exact in the half type, the FP32-storage run gives the
unrounded results of the same step, which numpy rounds here by the IEEE rule
(float16 cast; BF16 by integer round-to-nearest-even on the float32 bits).
A store that truncated would disagree on about half of the values; one that
rounded ties away from zero would disagree on the exact ties, which the
test counts and requires to be present."""
import numpy as np
import pytest

import paper_1902_11193_amd as P
from gpu_helpers import banner, W_LIB
from lbm_inputs import random_mask

pytestmark = pytest.mark.gpu

G = (1e-4, 0.0, 0.0)
E = 9  # FP16 storage exponent: values are stored as fp16(deviation * 2^9)


def bf16_round(x):
    """float64 values exact in float32 -> nearest-even BF16, as float64."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def f16_round(x):
    """float64 values exact in float32 -> nearest-even FP16 at scale 2^E."""
    return (np.asarray(x, np.float64) * 2.0**E).astype(np.float16).astype(np.float64) / 2.0**E


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_half_storage_rounds_to_nearest_even(storage):
    mask = random_mask((20, 24, 60), 0.3, 9)  # ~5e5 stored values: a few exact ties for BF16, dozens for FP16
    banner(f"codec rounding {storage}")
    rnd = bf16_round if storage == "bf16" else f16_round
    rng = np.random.default_rng(21)
    runs = {}
    for st in ("f32", storage):
        s = P.Solver(mask, 0.9, 3 / 16, "E", G, st)
        if st == "f16":
            s.set_storage_exponent(E)
        nf = s.n_fluid
        if "dev" not in runs:
            runs["dev"] = rnd(1e-3 * rng.standard_normal((19, nf)))  # exact in both storages
        s.set_state(W_LIB[:, None] + runs["dev"])
        s.step(1)
        runs[st] = s.get_state() - W_LIB[:, None]
        s.close()
    d32, dh = runs["f32"], runs[storage]
    assert np.array_equal(np.asarray(d32, np.float32).astype(np.float64), d32)  # FP32 results, exactly
    want = rnd(d32)
    assert np.array_equal(rnd(dh), dh)  # stored values are representable
    mism = dh != want
    other = rnd(2 * d32 - want)  # the neighbour on the far side of d32 (a value exactly halfway maps onto it)
    ties = int(np.count_nonzero((other != want) & (np.abs(want - d32) == np.abs(other - d32))))
    print(f"[codec] {storage}: {int(mism.sum())} of {mism.size} stored values differ from nearest-even "
          f"({ties} exact ties)", flush=True)
    # the two storages run the same FP32 arithmetic, so every value must match,
    # exact ties included (97 for BF16 and 647 for FP16 with these seeds)
    assert ties > 0
    assert not mism.any(), (storage, int(mism.sum()), mism.size)
