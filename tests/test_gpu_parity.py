"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

FP32 storage: the populations after 1, 2 and 50 steps from a random
non-equilibrium state agree with the oracle to 2e-6 of the deviation scale
(FP32 rounding of ~100 operations per step on values of that scale, 50 steps
of a contractive map).  The two neighbour layouts must agree bit for bit.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import paper_1902_11193_amd as P
from gpu_helpers import (banner, dense_from_lib, lib_from_dense, oracle_problem, random_state,
                         deviation_error, W_LIB)
from lbm_inputs import random_mask, sphere, percolating_x, gaussian_random_field, crop, workload

pytestmark = pytest.mark.gpu

CASES = [
    ("rand8", lambda: random_mask((8, 8, 8), 0.3, 11)),
    ("rand_ragged", lambda: random_mask((7, 9, 11), 0.35, 12)),
    ("rows130", lambda: random_mask((2, 3, 130), 0.25, 13)),
    ("sphere16", lambda: sphere(16, (7.5, 7.5, 7.5), 4.0)),
    # 300 planes: three 128-plane z-tiles in folded order, gathers across every tile face and the z wrap
    ("tiles300", lambda: random_mask((300, 3, 4), 0.3, 14)),
]
G = (1e-4, 5e-5, -2e-5)


def _run_pair(mask, rset, tau, Lam, index, nsteps_list, seed=0, g=G):
    s = P.Solver(mask, tau, Lam, rset, g, "f32", index)
    f0 = random_state(s.n_fluid, seed)
    s.set_state(f0)
    f0 = s.get_state()                      # FP32-rounded start, as the GPU holds it
    p = oracle_problem(mask, tau, Lam, rset, g)
    fh = dense_from_lib(p, f0)
    out = {}
    done = 0
    for n in nsteps_list:
        s.step(n - done)
        for _ in range(n - done):
            fh, u = p.step(fh)
        done = n
        out[n] = (s.get_state(), lib_from_dense(p, fh), s.mean_velocity(), p.mean_velocity(u).numpy())
    s.close()
    return out


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("index", ["table", "bitmap"])
def test_populations_match_oracle(name, make, index):
    mask = make()
    for rset, tau, Lam in (("E", 0.8, 3 / 16), ("SRT", 1.1, None), ("A", 0.9, None), ("B", 0.65, None),
                           ("C", 0.7, None), ("D", 1.3, None)):
        banner(f"populations {name} {index} {rset}")
        res = _run_pair(mask, rset, tau, Lam, index, [1, 2, 50])
        for n, (fg, fo, ug, uo) in res.items():
            err = deviation_error(fg, fo)
            assert err < 2e-6, (name, index, rset, n, err)
            assert np.allclose(ug, uo, rtol=0, atol=1e-6 * np.abs(uo).max()), (n, ug, uo)


@pytest.mark.parametrize("shape,solid", [((9, 10, 70), 0.3), ((5, 3, 18), 0.3), ((4, 7, 19), 0.2),
                                         ((6, 4, 37), 0.4), ((3, 1, 36), 0.1), ((3, 2, 4095), 0.05),
                                         ((260, 4, 5), 0.3)])
def test_table_and_bitmap_bitwise_equal(shape, solid):
    """The bitmap index reaches the same pull sources as the table: states and
    histories agree bit for bit, for row lengths around the bitmap's 18-voxel
    word step, a single-row-per-plane image, the longest rows it holds and
    three z-tiles (260 planes)."""
    mask = random_mask(shape, solid, 5)
    banner(f"table vs bitmap {shape}")
    states = []
    for index in ("table", "bitmap"):
        s = P.Solver(mask, 0.9, 1 / 12, "E", G, "f32", index)
        s.set_state(random_state(s.n_fluid, 3))
        s.step(20)
        states.append((s.get_state(), s.history(20)))
        s.close()
    assert np.array_equal(states[0][0], states[1][0])
    assert np.array_equal(states[0][1], states[1][1])


def test_deterministic_reruns():
    mask = random_mask((16, 16, 16), 0.35, 8)
    banner("determinism 16^3")
    runs = []
    for _ in range(2):
        s = P.Solver(mask, 1.0, 3 / 16, "E", (1e-5, 0, 0))
        s.step(100)
        runs.append((s.get_state(), s.history(100)))
        s.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


def test_mean_velocity_history_from_rest():
    mask = percolating_x(random_mask((12, 12, 12), 0.3, 9))
    banner("history from rest 12^3")
    s = P.Solver(mask, 0.9, 3 / 8, "E", (1e-5, 2e-6, 0))
    s.step(200)
    hg = s.history(200)
    p = oracle_problem(mask, 0.9, 3 / 8, "E", (1e-5, 2e-6, 0))
    ho = O.run(p, 200, keep_state=False)["umean"].numpy()
    assert np.abs(hg - ho).max() < 1e-6 * np.abs(ho).max()
    k = s.permeability()
    ko = p.permeability(torch.from_numpy(ho[-1])).numpy()
    assert abs(k[0] / ko[0] - 1) < 1e-6 and np.isnan(k[2])


def test_open_box_closed_form():
    """No solid: every step adds F to each node, <u>_n = (n - 1/2) g."""
    mask = np.zeros((5, 6, 70), np.uint8)
    banner("open box")
    g = (1e-5, -3e-6, 2e-6)
    s = P.Solver(mask, 0.7, None, "B", g)
    s.step(30)
    h = s.history(30)
    for n in range(1, 31):
        assert np.allclose(h[n - 1], (n - 0.5) * np.array(g), rtol=2e-6, atol=0)


def test_single_fluid_voxel_all_bounce_back():
    mask = np.ones((3, 3, 3), np.uint8)
    mask[1, 1, 1] = 0
    banner("single fluid voxel")
    for index in ("table", "bitmap"):
        s = P.Solver(mask, 1.0, 3 / 16, "E", (1e-3, 0, 0), index=index)
        assert s.n_fluid == 1
        f0 = random_state(1, 4)
        s.set_state(f0)
        f0 = s.get_state()
        s.step(7)
        p = oracle_problem(mask, 1.0, 3 / 16, "E", (1e-3, 0, 0))
        fh = dense_from_lib(p, f0)
        for _ in range(7):
            fh, _ = p.step(fh)
        assert deviation_error(s.get_state(), lib_from_dense(p, fh)) < 2e-6
        s.close()


def test_mass_is_conserved():
    mask = random_mask((16, 16, 16), 0.3, 2)
    banner("mass 16^3")
    s = P.Solver(mask, 0.8, 1 / 4, "E", (1e-4, 0, 0))
    s.step(2000)
    dm = s.mass_deviation()
    # FP32 rounding random walk: per node and step ~1e-11 on deviations ~1e-4
    assert abs(dm) < 1e-6 * s.n_fluid * 1e-4
    # total mass: n_fluid rho0 plus that deviation
    assert s.mass() == s.n_fluid + dm


def test_sc_sphere_permeability_matches_oracle_golden():
    """32^3 simple-cubic sphere array: k at equal step counts within 1e-6."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sc_sphere_32.json")))
    banner("sc_sphere_32 vs golden")
    m = workload("sc_sphere_32")
    for index in ("table", "bitmap"):
        s = P.Solver(m, 1.0, 3 / 16, "E", (1e-6, 0, 0), index=index)
        done = 0
        for n_str, ux in sorted(gold["umean_x"].items(), key=lambda kv: int(kv[0])):
            n = int(n_str)
            s.step(n - done)
            done = n
            assert abs(s.mean_velocity()[0] / ux - 1) < 1e-6, (index, n)
        k = s.permeability()[0]
        assert abs(k / gold["k_final"] - 1) < 1e-6
        s.close()


def test_run_to_steady_matches_oracle_step_count():
    """Same stopping rule as the oracle (per-step change of <u_x> below 1e-9,
    at most 5000 steps): same outcome and, at 5000 steps, the same k."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sc_sphere_32.json")))
    banner("run_to_steady sc_sphere_32")
    m = workload("sc_sphere_32")
    s = P.Solver(m, 1.0, 3 / 16, "E", (1e-6, 0, 0))
    r = s.run_to_steady(eps=1e-9, check_every=100, max_steps=5000)
    assert r["converged"] == gold["converged"]
    if gold["converged"]:
        assert gold["steps"] <= r["steps"] < gold["steps"] + 100
    else:
        assert r["steps"] == 5000
        assert abs(r["k"][0] / gold["k_final"] - 1) < 1e-6


def _record(name, **kw):
    """Print a measurement, and append it to storage_accuracy.jsonl in the
    directory LBM_RECORD_DIR names, when it is set."""
    line = json.dumps(dict(case=name, **kw))
    print(line)
    out = os.environ.get("LBM_RECORD_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "storage_accuracy.jsonl"), "a") as fh:
            fh.write(line + "\n")


@pytest.mark.parametrize("storage", ["f32", "f16r", "f16", "bf16"])
def test_reduced_storage_permeability(storage):
    """k after 600 steps with each storage type against the FP64 oracle on a
    32^3 crop of a porosity-0.2 Gaussian-random-field rock.  The crop is
    nearly blocked (k ~ 2e-3): density deviations exceed the velocity by ~1e3.
    FP32 storage is held to 1e-6 and FP16 relative to the per-node reference
    density (which rounds only the velocity-sized part) to the 1e-3 FP16
    target.  Plain FP16 and BF16 storage carry the density deviation in 11 and
    8 mantissa bits; their errors are measured and printed, not held to a
    bound."""
    rock = gaussian_random_field(64, 6.0, 0.2, seed=1904)
    m = crop(rock, 32)
    banner(f"reduced storage {storage} grf crop 32")
    N = 600
    p = oracle_problem(m, 1.0, 3 / 16, "E", (1e-6, 0, 0))
    ko = float(O.run(p, N, keep_state=False)["k"][0])
    s = P.Solver(m, 1.0, 3 / 16, "E", (1e-6, 0, 0), storage=storage)
    s.step(N)
    k = s.permeability()[0]
    rel = k / ko - 1
    print(f"[{storage}] crop32 k={k:.9g} oracle={ko:.9g} rel={rel:.3e}")
    _record("grf64 crop32, 600 steps", storage=storage, k=k, k_oracle=ko, rel=rel)
    assert np.isfinite(k)
    if storage == "f32":
        assert abs(rel) < 1e-6
    elif storage == "f16r":
        assert abs(rel) < 1e-3


@pytest.mark.parametrize("storage", ["f32", "f16r", "f16", "bf16"])
def test_grf_crop128_permeability_vs_oracle_golden(storage):
    """128^3 crop of the 512^3 rock: <u_x> after 500, 1000 and 2000 steps with
    each storage type against the FP64 oracle's values (tests/golden).  FP32
    storage is held to 1e-6; FP16 relative to the per-node reference density,
    the FP16-storage path this library offers for rock, to 1e-5 (the 1e-3
    target with margin; measured ~5e-6).  Plain FP16 and BF16 storage are
    measured and printed: in this poorly connected crop (k ~ 2e-2) pressure
    builds up in dead ends until the density deviation is ~1e3 times the flow
    signal, which 11 or 8 mantissa bits cannot carry alongside it."""
    path = os.path.join(os.path.dirname(__file__), "golden", "grf_crop128.json")
    gold = json.load(open(path))
    m = crop(workload("grf_512"), 128)
    banner(f"grf crop128 {storage}")
    s = P.Solver(m, 1.0, 3 / 16, "E", (1e-6, 0, 0), storage=storage)
    assert s.n_fluid == gold["n_fluid"]
    done = 0
    errs = {}
    for n_str, ux in sorted(gold["umean_x"].items(), key=lambda kv: int(kv[0])):
        n = int(n_str)
        s.step(n - done)
        done = n
        rel = s.mean_velocity()[0] / ux - 1
        print(f"[{storage}] crop128 n={n} rel={rel:.3e}")
        errs[n] = float(rel)
    _record("grf_512 crop128", storage=storage, rel_by_step=errs)
    assert all(np.isfinite(list(errs.values())))
    worst = max(abs(v) for v in errs.values())
    if storage == "f32":
        assert worst < 1e-6
    elif storage == "f16r":
        assert worst < 1e-5


def test_force_field_uniform_equals_default():
    mask = random_mask((10, 11, 12), 0.3, 6)
    banner("force field")
    g = (2e-5, -1e-5, 3e-6)
    a = P.Solver(mask, 0.9, 1 / 12, "E", g)
    a.step(30)
    b = P.Solver(mask, 0.9, 1 / 12, "E", g)
    fld = torch.tensor(np.array(g, np.float32)[:, None].repeat(b.n_fluid, 1), device="cuda")
    b.set_force_field(fld)
    b.step(30)
    # the per-node force is loaded instead of passed as a constant: the same
    # arithmetic up to the compiler's FP32 contraction choices
    assert deviation_error(a.get_state(), b.get_state()) < 1e-6


def test_force_field_matches_oracle():
    mask = random_mask((8, 9, 10), 0.3, 7)
    banner("force field vs oracle")
    rng = np.random.default_rng(3)
    s = P.Solver(mask, 1.1, None, "D", (1e-4, 0, 0))
    gf = (1e-4 * (1 + 0.5 * rng.standard_normal((3, s.n_fluid)))).astype(np.float32)
    s.set_force_field(torch.from_numpy(gf).cuda())
    s.step(40)
    dense = np.zeros((3,) + mask.shape)
    dense.reshape(3, -1)[:, P.lbm_node_order(mask)] = gf.astype(np.float64)
    p = O.Problem(mask, 1.1, None, "D", (1e-4, 0, 0), g_field=dense)
    r = O.run(p, 40)
    assert deviation_error(s.get_state(), lib_from_dense(p, r["state"])) < 2e-6


def test_storage_exponent_roundtrip():
    mask = random_mask((8, 8, 8), 0.3, 1)
    banner("fp16 exponent")
    s = P.Solver(mask, 1.0, 3 / 16, "E", (1e-4, 0, 0), storage="f16")
    s.step(10)
    f1 = s.get_state()
    s.set_storage_exponent(5)
    f2 = s.get_state()
    assert np.abs(f1 - f2).max() < 1e-3 * np.abs(f1 - W_LIB[:, None]).max()


def test_sampled_full_size_step_grf_512():
    """512^3 porosity-0.2 rock at full size, bench launch configuration:
    one step checked at sampled nodes against the oracle's collision."""
    m = workload("grf_512")
    banner("grf_512 sampled step")
    s = P.Solver(m, 1.0, 3 / 16, "E", (1e-6, 0, 0))
    s.step(20)
    f20 = s.get_state()
    s.step(1)
    f21 = s.get_state()
    nf = s.n_fluid
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(nf, 4096, replace=False))
    t = P.lbm_neighbor_table(m)[:, sample]            # (18, S) pull sources
    c = P.lbm_velocities()
    f = np.empty((19, len(sample)))
    f[0] = f20[0, sample]
    for i in range(1, 19):
        j = i + 1 if i % 2 else i - 1
        src = t[i - 1]
        f[i] = np.where(src >= 0, f20[i, np.maximum(src, 0)], f20[j, sample])
    lat = O.Lattice.make()
    from gpu_helpers import PERM
    fo = torch.from_numpy(f[PERM])
    F = torch.tensor([[1e-6], [0.0], [0.0]], dtype=torch.float64).expand(3, len(sample))
    out = O.collide(fo, O.rates("E", 1.0, 3 / 16), F, lat).numpy()
    want = np.empty_like(out)
    want[PERM] = out
    got = f21[:, sample]
    assert deviation_error(got, want) < 2e-6
    assert abs(s.mass_deviation()) < 1e-3 * nf * 1e-6
    del c


def test_pack256_crop64_matches_oracle():
    """The 256^3 sphere pack's 64^3 corner crop (re-filtered for x-spanning
    fluid): k after 50 and 200 steps from rest against the FP64 oracle, for
    Set E at the ends of the pack study's relaxation times."""
    m = crop(workload("pack_256"), 64)
    for tau in (0.6, 1.3):
        banner(f"pack256 crop64 tau={tau}")
        p = oracle_problem(m, tau, 3 / 16, "E", (1e-6, 0, 0))
        r = O.run(p, 200, keep_state=False)
        s = P.Solver(m, tau, 3 / 16, "E", (1e-6, 0, 0))
        s.step(50)
        k50 = s.permeability()[0]
        s.step(150)
        k200 = s.permeability()[0]
        ko50 = float(p.permeability(r["umean"][49])[0])
        ko200 = float(r["k"][0])
        assert abs(k50 / ko50 - 1) < 1e-6 and abs(k200 / ko200 - 1) < 1e-6, (tau, k50, ko50, k200, ko200)
        s.close()
