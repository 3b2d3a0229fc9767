"""The 1024^3 rock (porosity 0.134 after filtering, 144,228,832 fluid nodes,
states of 11 GB in FP32) at full size, with each storage type: one step at
4096 sampled nodes against the oracle's collision, read through
lbm_get_state_nodes.  At this size the
population arrays exceed 4 GiB, so the per-chunk 32-bit gather offsets are
exercised where they matter."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1902_11193_amd as P
from gpu_helpers import PERM, W_LIB, banner, deviation_error
from lbm_inputs import workload

pytestmark = pytest.mark.gpu

G = 1e-7


@pytest.fixture(scope="module")
def rock():
    banner("generating grf_1024")
    return workload("grf_1024")


def _oracle_step(f_src, sample, t, fo_of):
    """Gathered populations of the sampled nodes from the states of their
    sources, then the oracle's collision."""
    f = np.empty((19, len(sample)))
    f[0] = fo_of(sample)[0]
    for i in range(1, 19):
        j = i + 1 if i % 2 else i - 1
        src = t[i - 1]
        pulled = fo_of(np.where(src >= 0, src, sample))[i]   # wall entries are not used
        own = fo_of(sample)[j]
        f[i] = np.where(src >= 0, pulled, own)
    lat = O.Lattice.make()
    F = torch.tensor([[G], [0.0], [0.0]], dtype=torch.float64).expand(3, len(sample))
    out = O.collide(torch.from_numpy(f[PERM]), O.rates("E", 1.0, 3 / 16), F, lat).numpy()
    want = np.empty_like(out)
    want[PERM] = out
    return want


@pytest.mark.parametrize("storage,collision", [("f32", "mrt"), ("f16r", "mrt"), ("f16", "mrt"), ("bf16", "mrt"),
                                               ("f32", "trt")])
def test_sampled_step_grf_1024(rock, storage, collision):
    """(Set E is a two-rate set, so the link-wise TRT kernel computes the
    oracle's moment-space collision too.)"""
    banner(f"grf_1024 sampled step {storage} {collision}")
    s = P.Solver(rock, 1.0, 3 / 16, "E", (G, 0, 0), storage, "bitmap")
    s.set_collision(collision)
    nf = s.n_fluid
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(nf, 4096, replace=False))
    t = P.lbm_neighbor_nodes(rock, sample)                      # (18, S)
    needed = np.unique(np.concatenate([sample, t[t >= 0].astype(np.int64)]))
    s.step(20)
    f20 = s.get_state_nodes(needed)
    pos = {int(n): k for k, n in enumerate(needed)}
    fo_of = lambda nodes: f20[:, [pos[int(n)] for n in nodes]]
    s.step(1)
    got = s.get_state_nodes(sample)
    want = _oracle_step(f20, sample, t, fo_of)
    print(f"[fullsize] {storage} {collision}: max error / deviation scale {deviation_error(got, want):.3e}",
          flush=True)
    if storage == "f32":
        assert deviation_error(got, want) < 2e-6
    elif storage == "f16r":
        # FP16 rounds the part left after the reference density
        small = want - W_LIB[:, None] * want.sum(0)[None, :]
        assert np.abs(got - want).max() < 2e-3 * np.abs(small).max()
    else:
        # the stored deviation is rounded to 11 (FP16) or 8 (BF16) significant bits
        bound = 2.0**-10 if storage == "f16" else 2.0**-7
        assert deviation_error(got, want) < bound
    assert np.isfinite(s.mass_deviation())
    s.close()
    del s
    torch.cuda.empty_cache()
