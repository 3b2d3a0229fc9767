"""GPU parity of the non-periodic image boundaries (Sec. 2.3): full-way
bounce-back against the oracle's full-way stream, and the padded / mirrored
image (lbm_boundary_image) against the oracle's symmetry planes on the
original image.  FP32 storage, 2e-6 of the deviation scale as in the other
population tests."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1902_11193_amd as P
from gpu_helpers import banner, dense_from_lib, lib_from_dense, random_state, deviation_error, W_LIB
from lbm_inputs import random_mask, sphere

pytestmark = pytest.mark.gpu

G = (1e-4, 5e-5, -2e-5)


@pytest.mark.parametrize("name,make", [("rand8", lambda: random_mask((8, 8, 8), 0.3, 11)),
                                       ("rand_ragged", lambda: random_mask((7, 9, 11), 0.35, 12)),
                                       ("sphere16", lambda: sphere(16, (7.5, 7.5, 7.5), 4.0))])
@pytest.mark.parametrize("index", ["table", "bitmap"])
@pytest.mark.parametrize("collision", ["mrt", "trt"])
def test_fullway_bounce_back_matches_oracle(name, make, index, collision):
    mask = make()
    banner(f"fullway {name} {index} {collision}")
    s = P.Solver(mask, 0.9, 3 / 16, "E", G, "f32", index)
    s.set_collision(collision)
    s.set_wall("fullway")
    f0 = random_state(s.n_fluid, 5)
    s.set_state(f0)                     # the one-step-older state starts equal to it
    f0 = s.get_state()
    p = O.Problem(mask, 0.9, 3 / 16, "E", G, fullway=True, collision=collision)
    d0 = dense_from_lib(p, f0)
    fh = torch.stack([d0, d0.clone()])
    done = 0
    for n in (1, 2, 50):
        s.step(n - done)
        for _ in range(n - done):
            fh, u = p.step(fh)
        done = n
        err = deviation_error(s.get_state(), lib_from_dense(p, fh[0]))
        assert err < 2e-6, (name, index, n, err)
        uo = p.mean_velocity(u).numpy()
        assert np.allclose(s.mean_velocity(), uo, rtol=0, atol=1e-6 * np.abs(uo).max())
    s.close()


def test_fullway_steady_k_equals_halfway():
    mask = random_mask((8, 8, 8), 0.3, 11)
    banner("fullway steady k 8^3")
    ks = []
    for wall in ("halfway", "fullway"):
        s = P.Solver(mask, 1.0, 3 / 16, "E", (1e-5, 0, 0), "f32", "bitmap")
        s.set_wall(wall)
        s.step(4000)
        ks.append(float(s.history(2)[:, 0].mean()))   # two-step mean: immune to a period-2 mode
        s.close()
    assert abs(ks[1] / ks[0] - 1) < 1e-5, ks


@pytest.mark.parametrize("pad,sym", [(0, "yz"), (2, "yz"), (3, "y"), (0, "z")])
def test_mirrored_image_matches_oracle_symmetry_planes(pad, sym):
    """The library on the padded, mirrored image (periodic) equals the oracle
    with symmetry planes on the padded original, on the original quarter."""
    mask = random_mask((6, 7, 9), 0.3, 21)
    banner(f"mirror pad={pad} sym={sym}")
    big = P.lbm_boundary_image(mask, pad, "y" in sym, "z" in sym)
    padded = np.pad(mask, ((0, 0), (0, 0), (pad, pad)))
    s = P.Solver(big, 0.9, 3 / 16, "E", (1e-4, 0, 0), "f32", "bitmap")
    pbig = O.Problem(big, 0.9, 3 / 16, "E", (1e-4, 0, 0))        # only for the node-order map
    p = O.Problem(padded, 0.9, 3 / 16, "E", (1e-4, 0, 0), symmetric=sym)
    fh = p.initial()
    nz, ny, _ = padded.shape
    done = 0
    for n in (1, 2, 50):
        s.step(n - done)
        for _ in range(n - done):
            fh, u = p.step(fh)
        done = n
        got = dense_from_lib(pbig, s.get_state())[:, :nz, :ny, :]
        ref = lib_from_dense(p, fh)
        err = deviation_error(lib_from_dense(p, got), ref)
        assert err < 2e-6, (pad, sym, n, err)
        # the driven superficial velocity of the big box is that of the quarter
        assert abs(float(s.mean_velocity()[0]) / float(p.mean_velocity(u)[0]) - 1) < 1e-5
    s.close()


def test_wall_mode_errors():
    mask = random_mask((6, 6, 6), 0.3, 2)
    banner("wall mode errors")
    s = P.Solver(mask, 0.9, 3 / 16, "E", G, "f16", "bitmap")
    with pytest.raises(P.LbmError) as e:
        s.set_wall("fullway")
    assert e.value.code == P.LBM_EINVAL
    s.close()
    s = P.Solver(mask, 0.9, 3 / 16, "E", (1e-5, 0, 0), "f32", "bitmap")
    s.set_wall("fullway")
    with pytest.raises(P.LbmError) as e:
        s.adjoint(10, 5)
    assert e.value.code == P.LBM_EINVAL
    s.set_wall("halfway")
    s.step(2)
    s.close()


@pytest.mark.parametrize("name,make", [("rand_x12", lambda: random_mask((6, 7, 12), 0.3, 31)),
                                       ("slit", lambda: __import__("lbm_inputs").slit(10, 9, 3, 6))])
@pytest.mark.parametrize("collision", ["mrt", "trt"])
def test_pressure_faces_match_oracle(name, make, collision):
    """Zou-He pressure inlet/outlet on the x faces against the oracle's."""
    mask = make()
    banner(f"pressure {name} {collision}")
    rin, rout = 1 + 5e-5, 1 - 5e-5
    s = P.Solver(mask, 0.9, 3 / 16, "E", (0.0, 0.0, 0.0), "f32", "bitmap")
    s.set_collision(collision)
    s.set_pressure(rin, rout)
    f0 = random_state(s.n_fluid, 9, amp=1e-5)
    s.set_state(f0)
    f0 = s.get_state()
    p = O.Problem(mask, 0.9, 3 / 16, "E", (0, 0, 0), collision=collision, pressure=(rin, rout))
    fh = dense_from_lib(p, f0)
    done = 0
    for n in (1, 2, 50):
        s.step(n - done)
        for _ in range(n - done):
            fh, u = p.step(fh)
        done = n
        err = deviation_error(s.get_state(), lib_from_dense(p, fh))
        assert err < 2e-6, (name, n, err)
        kg, ko = float(s.permeability()[0]), float(p.permeability(p.mean_velocity(u))[0])
        assert abs(kg - ko) <= 1e-5 * abs(ko) + 1e-12, (n, kg, ko)
    s.close()


def test_pressure_driven_slit_permeability():
    """At Lambda = 1/4 the pressure-driven slit reaches the closed form."""
    from lbm_inputs import slit

    banner("pressure slit k")
    H, Ly = 8, 10
    s = P.Solver(slit(12, Ly, 1, H), 0.8, 1 / 4, "E", (0.0, 0.0, 0.0), "f32", "bitmap")
    s.set_pressure(1 + 5e-5, 1 - 5e-5)
    r = s.run_to_steady(eps=1e-9, check_every=100, max_steps=20000)
    k_exact = H * (H * H - 1 + 8 / 4) / (12 * Ly)
    assert abs(float(r["k"][0]) / k_exact - 1) < 1e-4, (r, k_exact)
    s.close()


def test_pressure_mode_errors():
    mask = random_mask((6, 6, 6), 0.3, 2)
    banner("pressure errors")
    for storage, index, g in (("f16", "bitmap", (0, 0, 0)), ("f32", "table", (0, 0, 0)),
                              ("f32", "bitmap", (1e-6, 0, 0))):
        s = P.Solver(mask, 0.9, 3 / 16, "E", g, storage, index)
        with pytest.raises(P.LbmError) as e:
            s.set_pressure(1.001, 0.999)
        assert e.value.code == P.LBM_EINVAL
        s.close()
    s = P.Solver(mask, 0.9, 3 / 16, "E", (0, 0, 0), "f32", "bitmap")
    with pytest.raises(P.LbmError):
        s.set_pressure(1.0, 1.0)
    s.set_pressure(1.001, 0.999)
    with pytest.raises(P.LbmError):
        s.adjoint(10, 5)
    s.set_pressure(None)
    s.close()


def test_fullway_last_node_with_many_chunks_per_block():
    """Full-way bounce-back on an image large enough that every block walks
    several chunks (waves of a block drift apart), with the last node of the
    list on a wall link and the lanes past the list filling later waves of the
    last chunk: they must not touch that node's delay-line or state slots."""
    mask = random_mask((100, 104, 112), 0.1, 7)
    order = P.lbm_node_order(mask)
    nz, ny, nx = mask.shape
    last = int(order[-1])
    x, y, z = last % nx, (last // nx) % ny, last // (nx * ny)
    mask[z, y, (x + 1) % nx] = 1                 # a wall link at the last node
    # drop fluid voxels from the front of the list until 70 lanes of the last
    # chunk are live: node nf-1 in wave 1, waves 2 and 3 past the list
    nf = int(np.count_nonzero(mask == 0))
    drop = (nf - 70) % 256
    front = P.lbm_node_order(mask)[:drop]
    mask.reshape(-1)[front] = 1
    nf = int(np.count_nonzero(mask == 0))
    assert nf % 256 == 70 and int(P.lbm_node_order(mask)[-1]) == last
    banner(f"fullway many chunks per block, nf={nf}")
    s = P.Solver(mask, 0.9, 3 / 16, "E", G, "f32", "bitmap")
    s.set_wall("fullway")
    f0 = random_state(s.n_fluid, 9)
    s.set_state(f0)
    f0 = s.get_state()
    p = O.Problem(mask, 0.9, 3 / 16, "E", G, fullway=True)
    d0 = dense_from_lib(p, f0)
    fh = torch.stack([d0, d0.clone()])
    done = 0
    for n in (1, 2, 50):
        s.step(n - done)
        for _ in range(n - done):
            fh, _ = p.step(fh)
        done = n
        got, ref = s.get_state(), lib_from_dense(p, fh[0])
        err_last = deviation_error(got[:, -1:], ref[:, -1:])
        err = deviation_error(got, ref)
        print(f"step {n}: last node {err_last:.2e}, all nodes {err:.2e}", flush=True)
        assert err_last < 2e-6 and err < 2e-6, (n, err_last, err)
    s.close()


@pytest.mark.parametrize("shape,sym", [((6, 7, 13), "y"), ((6, 7, 13), "z"), ((6, 7, 13), "yz"),
                                       ((2, 3, 11), "yz"), ((5, 1, 9), "y")])
@pytest.mark.parametrize("wall", ["halfway", "fullway"])
@pytest.mark.parametrize("collision", ["mrt", "trt"])
def test_symmetry_planes_in_kernel_match_oracle(shape, sym, wall, collision):
    """lbm_set_symmetry (mirror planes applied in the step kernel, Sec. 2.3)
    against the oracle's symmetry planes on the same padded image, from a
    random state, 1, 2 and 50 steps; thin boxes where one row or plane is both
    faces included."""
    mask = np.pad(random_mask(shape, 0.3, 21), ((0, 0), (0, 0), (2, 2)))
    banner(f"symmetry planes in kernel {shape} {sym} {wall} {collision}")
    s = P.Solver(mask, 0.9, 3 / 16, "E", G, "f32", "bitmap")
    s.set_symmetry("y" in sym, "z" in sym)
    s.set_collision(collision)
    if wall == "fullway":
        s.set_wall("fullway")
    f0 = random_state(s.n_fluid, 6)
    s.set_state(f0)
    f0 = s.get_state()
    p = O.Problem(mask, 0.9, 3 / 16, "E", G, symmetric=sym, fullway=wall == "fullway", collision=collision)
    d0 = dense_from_lib(p, f0)
    fh = torch.stack([d0, d0.clone()]) if wall == "fullway" else d0
    done = 0
    for n in (1, 2, 50):
        s.step(n - done)
        for _ in range(n - done):
            fh, u = p.step(fh)
        done = n
        ref = lib_from_dense(p, fh[0] if wall == "fullway" else fh)
        err = deviation_error(s.get_state(), ref)
        assert err < 2e-6, (shape, sym, wall, collision, n, err)
        # <u> sums momenta made of deviations of the random state's scale:
        # its FP32 error is bounded on that scale, not on <u>'s own (~1e-2 of it)
        uo = p.mean_velocity(u).numpy()
        assert np.allclose(s.mean_velocity(), uo, rtol=0, atol=2e-6 * np.abs(ref - W_LIB[:, None]).max())
    s.close()


def test_symmetry_planes_with_force_field_match_oracle():
    mask = np.pad(random_mask((7, 8, 10), 0.3, 22), ((0, 0), (0, 0), (3, 3)))
    banner("symmetry planes with a force field")
    rng = np.random.default_rng(5)
    s = P.Solver(mask, 1.1, None, "B", (1e-4, 0, 0), "f32", "bitmap")
    s.set_symmetry(True, True)
    gf = (1e-4 * (1 + 0.5 * rng.standard_normal((3, s.n_fluid)))).astype(np.float32)
    s.set_force_field(torch.from_numpy(gf).cuda())
    s.step(40)
    dense = np.zeros((3,) + mask.shape)
    dense.reshape(3, -1)[:, P.lbm_node_order(mask)] = gf.astype(np.float64)
    p = O.Problem(mask, 1.1, None, "B", (1e-4, 0, 0), g_field=dense, symmetric="yz")
    r = O.run(p, 40)
    assert deviation_error(s.get_state(), lib_from_dense(p, r["state"])) < 2e-6
    s.close()


def test_symmetry_planes_equal_the_reflected_image():
    """The paper's sphere-pack setup (5 padding layers, mirror planes on the
    lateral faces) on a 32^3 crop of the 128^3 pack: k from the in-kernel
    symmetry planes equals k of the reflected periodic image (4x the nodes)
    at equal step counts."""
    from lbm_inputs import crop, workload
    m = crop(workload("pack_128"), 32)
    banner("symmetry planes vs reflected image, pack_128 crop 32")
    padded = np.pad(m, ((0, 0), (0, 0), (5, 5)))
    a = P.Solver(padded, 1.0, 3 / 16, "E", (1e-6, 0, 0), "f32", "bitmap")
    a.set_symmetry(True, True)
    big = P.lbm_boundary_image(m, 5, True, True)
    b = P.Solver(big, 1.0, 3 / 16, "E", (1e-6, 0, 0), "f32", "bitmap")
    assert b.n_fluid == 4 * a.n_fluid
    for n in (100, 400):
        a.step(n - a.steps_done)
        b.step(n - b.steps_done)
        ka, kb = a.permeability()[0], b.permeability()[0]
        print(f"n={n}: k symmetry planes {ka:.9g}, reflected image {kb:.9g}")
        assert abs(ka / kb - 1) < 1e-6
    a.close()
    b.close()


def test_symmetry_plane_argument_errors():
    mask = np.pad(random_mask((6, 7, 9), 0.3, 23), ((0, 0), (0, 0), (2, 2)))
    banner("symmetry plane argument errors")
    for storage, index in (("f32", "table"), ("f16", "bitmap"), ("f16r", "bitmap")):
        s = P.Solver(mask, 0.9, 3 / 16, "E", (1e-4, 0, 0), storage, index)
        with pytest.raises(P.LbmError) as e:
            s.set_symmetry(True, False)
        assert e.value.code == P.LBM_EINVAL
        s.close()
    s = P.Solver(mask, 0.9, 3 / 16, "E", (0, 0, 0), "f32", "bitmap")
    s.set_pressure(1.001, 1.0)
    with pytest.raises(P.LbmError):
        s.set_symmetry(False, True)
    s.set_pressure(None)
    s.set_symmetry(False, True)
    with pytest.raises(P.LbmError):
        s.set_pressure(1.001, 1.0)
    s.close()
    s = P.Solver(mask, 0.9, 3 / 16, "E", (1e-4, 0, 0), "f32", "bitmap")
    s.set_symmetry(True, True)
    with pytest.raises(P.LbmError):
        s.adjoint(10, 5)
    s.set_symmetry(False, False)      # back to the periodic box: the adjoint runs
    assert np.isfinite(s.adjoint(10, 5)["k"])
    s.close()
