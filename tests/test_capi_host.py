"""Host-side checks of the C-ABI library: loads, exports what include/lbm.h
declares, host logic (rates, neighbour table) and argument validation.  No
call here reaches the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1902_11193_amd as P
from lbm_inputs import random_mask, sphere, slit

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "lbm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(P.SIGNATURES) == names


def test_velocity_order_matches_header_and_pairs():
    c = P.lbm_velocities()
    txt = open(HEADER).read()
    doc = [tuple(int(v) for v in m) for m in re.findall(r"\d+:\(\s*(-?\d),\s*(-?\d),\s*(-?\d)\)", txt)]
    assert [tuple(r) for r in c] == doc[:19]
    for i in range(1, 19, 2):
        assert np.array_equal(c[i], -c[i + 1])
    oc = {tuple(v.tolist()) for v in O.velocities()}
    assert {tuple(r) for r in c} == oc


@pytest.mark.parametrize("rset", list(P.SETS))
@pytest.mark.parametrize("tau_key", ["0.6", "1.3"])
def test_rates_equal_table2_entries(rset, tau_key):
    """lbm_rates against Table 2 evaluated by hand (tests/golden/paper_values.json)."""
    import json
    from fractions import Fraction
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))["table2_rates"]
    want = [float(Fraction(v)) for v in gold["rates"][tau_key][rset]]
    s, _, _ = P.lbm_rates(rset, float(tau_key), float(Fraction(gold["Lambda_E"])))
    assert np.allclose(s, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("rset", list(P.SETS))
@pytest.mark.parametrize("tau", [0.6, 1.0, 1.37])
def test_rates_match_oracle_and_derivatives(rset, tau):
    Lam = 0.21
    s, dt, dl = P.lbm_rates(rset, tau, Lam)
    want = O.rates(rset, tau, Lam if rset == "E" else None).numpy()
    assert np.allclose(s, want, rtol=0, atol=1e-15)
    h = 1e-6
    sp, _, _ = P.lbm_rates(rset, tau + h, Lam)
    sm, _, _ = P.lbm_rates(rset, tau - h, Lam)
    assert np.allclose(dt, (sp - sm) / (2 * h), atol=1e-8)
    if rset == "E":
        sp, _, _ = P.lbm_rates(rset, tau, Lam + h)
        sm, _, _ = P.lbm_rates(rset, tau, Lam - h)
        assert np.allclose(dl, (sp - sm) / (2 * h), atol=1e-8)
    else:
        assert not dl.any()


def test_rates_reject():
    for args in (("E", 0.5, 0.2), ("E", 1.0, 0.0), (7, 1.0, 0.2), ("SRT", float("nan"), 0.2)):
        with pytest.raises(P.LbmError) as e:
            P.lbm_rates(*args)
        assert e.value.code == P.LBM_EINVAL


def _brute_node_order(mask, tile=128):
    """Fluid voxels sorted by (position of the z-tile, y, z % tile, x), where the
    tiles t = z // tile of T are folded into the order 0, T-1, 1, T-2, ...
    An image whose gathers span less than 2^32 bytes around every chunk with
    128-plane tiles (every image of these tests) gets tiles of 128 planes."""
    nz, ny, nx = mask.shape
    T = -(-nz // tile)
    t = np.arange(T)
    pos = np.where(2 * t < T, 2 * t, 2 * (T - 1 - t) + 1)
    assert np.array_equal(np.sort(pos), t)
    fl = np.flatnonzero(mask.reshape(-1) == 0)
    z, y, x = np.unravel_index(fl, mask.shape)
    key = np.lexsort((x, z % tile, y, pos[z // tile]))
    return fl[key]


def _brute_table(mask):
    nz, ny, nx = mask.shape
    c = P.lbm_velocities()
    fl = _brute_node_order(mask)
    node = -np.ones(mask.size, np.int64)
    node[fl] = np.arange(len(fl))
    z, y, x = np.unravel_index(fl, mask.shape)
    t = np.empty((18, len(fl)), np.int64)
    for i in range(1, 19):
        sx, sy, sz = (x - c[i, 0]) % nx, (y - c[i, 1]) % ny, (z - c[i, 2]) % nz
        t[i - 1] = node[np.ravel_multi_index((sz, sy, sx), mask.shape)]
    return t


@pytest.mark.parametrize("shape,sf,seed", [((5, 6, 7), 0.3, 0), ((8, 8, 8), 0.5, 1), ((1, 9, 70), 0.2, 2),
                                           ((3, 2, 130), 0.4, 3)])
def test_neighbor_table_brute_force_and_permutation(shape, sf, seed):
    mask = random_mask(shape, sf, seed)
    if (mask == 0).sum() == 0:
        mask.flat[0] = 0
    t = P.lbm_neighbor_table(mask)
    assert np.array_equal(t, _brute_table(mask))
    # every post-collision value (j, m) is read exactly once by the pull + bounce-back
    nf = t.shape[1]
    reads = np.zeros((19, nf), np.int64)
    reads[0] += 1
    for i in range(1, 19):
        j = i + 1 if i % 2 else i - 1
        src = t[i - 1]
        ok = src >= 0
        np.add.at(reads[i], src[ok], 1)
        np.add.at(reads[j], np.flatnonzero(~ok), 1)
    assert (reads == 1).all()


@pytest.mark.parametrize("shape", [(5, 6, 7), (40, 3, 9), (33, 17, 2), (64, 2, 3), (70, 3, 4), (300, 2, 3),
                                   (390, 3, 2), (129, 2, 2)])
def test_node_order_is_z_tiled_rows(shape):
    mask = random_mask(shape, 0.3, 4)
    order = P.lbm_node_order(mask)
    assert np.array_equal(order, _brute_node_order(mask))
    assert np.array_equal(np.sort(order), np.flatnonzero(mask.reshape(-1) == 0))
    perm = P.raster_permutation(mask)
    assert np.array_equal(np.flatnonzero(mask.reshape(-1) == 0)[perm], order)


def test_workspace_query_counts_and_errors():
    m = sphere(16, (7.5, 7.5, 7.5), 4.0)
    nb, nf = P.lbm_workspace_query(m, "f32", "table")
    assert nf == int((m == 0).sum())
    nb16, _ = P.lbm_workspace_query(m, "f16", "bitmap")
    assert nb16 < nb
    with pytest.raises(P.LbmError) as e:
        P.lbm_workspace_query(np.ones((4, 4, 4), np.uint8))
    assert e.value.code == P.LBM_ENOFLUID
    L = P.lib()
    g = np.zeros((2, 2, 2), np.uint8)
    ptr = g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    nbytes, n = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert L.lbm_workspace_query(ptr, 0, 2, 2, 0, 0, ctypes.byref(nbytes), ctypes.byref(n)) == P.LBM_EINVAL
    assert L.lbm_workspace_query(ptr, 2, 2, 2, 4, 0, ctypes.byref(nbytes), ctypes.byref(n)) == P.LBM_EINVAL
    assert L.lbm_workspace_query(ptr, 2, 2, 2, 0, 2, ctypes.byref(nbytes), ctypes.byref(n)) == P.LBM_EINVAL
    assert L.lbm_workspace_query(None, 2, 2, 2, 0, 0, ctypes.byref(nbytes), ctypes.byref(n)) == P.LBM_EINVAL


def test_bitmap_row_length_limit():
    """The bitmap index takes rows of up to 4095 voxels (its 18-bit row-base
    differences and 16-bit count fields are sized for them); longer ones are
    refused (LBM_ERANGE) and the table index takes them."""
    for nx, ok in ((4095, True), (4096, False)):
        m = np.zeros((1, 1, nx), np.uint8)
        if ok:
            nb, nf = P.lbm_workspace_query(m, "f16", "bitmap")
            assert nf == nx and nb > 0
        else:
            with pytest.raises(P.LbmError) as e:
                P.lbm_workspace_query(m, "f16", "bitmap")
            assert e.value.code == P.LBM_ERANGE
            assert b"4095" in P.lib().lbm_last_error()
        assert P.lbm_workspace_query(m, "f16", "table")[1] == nx


def _setup_rc(mask, tau=1.0, Lam=0.1875, rset=5, g=(1e-6, 0, 0), storage=0, index=1, ws=None, nbytes=None,
              fn="lbm_setup"):
    """Call lbm_setup (or lbm_setup_static) with a fake (never dereferenced)
    workspace; validation fails first."""
    L = P.lib()
    m = np.ascontiguousarray(mask, np.uint8)
    nz, ny, nx = m.shape
    ctx = ctypes.c_void_p()
    gv = (ctypes.c_double * 3)(*g)
    rc = getattr(L, fn)(ctypes.byref(ctx), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), nx, ny, nz, tau, Lam,
                        rset, gv, storage, index, ws, nbytes if nbytes is not None else 0, None)
    assert not ctx.value
    return rc


def test_setup_validates_before_any_device_call():
    m = slit(4, 6, 4, 3)
    fake = ctypes.c_void_p(4096)  # aligned, never touched: every case fails validation first
    assert _setup_rc(m, tau=0.5, ws=fake, nbytes=1 << 40) == P.LBM_EINVAL
    assert _setup_rc(m, tau=float("inf"), ws=fake, nbytes=1 << 40) == P.LBM_EINVAL
    assert _setup_rc(m, rset=6, ws=fake, nbytes=1 << 40) == P.LBM_EINVAL
    assert _setup_rc(m, Lam=0.0, ws=fake, nbytes=1 << 40) == P.LBM_EINVAL
    assert _setup_rc(m, g=(float("nan"), 0, 0), ws=fake, nbytes=1 << 40) == P.LBM_EINVAL
    assert _setup_rc(m, storage=5, ws=fake, nbytes=1 << 40) == P.LBM_EINVAL
    assert _setup_rc(np.ones((3, 3, 3)), ws=fake, nbytes=1 << 40) == P.LBM_ENOFLUID
    assert _setup_rc(m, ws=None, nbytes=1 << 40) == P.LBM_EWORKSPACE
    assert _setup_rc(m, ws=fake, nbytes=16) == P.LBM_EWORKSPACE
    assert _setup_rc(m, ws=ctypes.c_void_p(4096 + 8), nbytes=1 << 40) == P.LBM_EWORKSPACE
    assert b"workspace" in P.lib().lbm_last_error()


def test_setup_static_validates_and_needs_less_workspace():
    """lbm_setup_static checks its arguments as lbm_setup does, before any
    device call, and sizes the workspace without the reduction scratch."""
    m = slit(4, 6, 4, 3)
    fake = ctypes.c_void_p(4096)
    hdr = open(HEADER).read()
    assert f"#define LBM_REDUCTION_BYTES {P.LBM_REDUCTION_BYTES}" in hdr
    assert f"#define LBM_EBUSY ({P.LBM_EBUSY})" in hdr
    for bad in (dict(tau=0.5), dict(rset=6), dict(storage=5), dict(g=(float("nan"), 0, 0))):
        assert _setup_rc(m, ws=fake, nbytes=1 << 40, fn="lbm_setup_static", **bad) == P.LBM_EINVAL
    nbytes, _ = P.lbm_workspace_query(m, "f32", "bitmap")
    need = nbytes - P.LBM_REDUCTION_BYTES
    assert need > 0
    assert _setup_rc(m, ws=fake, nbytes=need - 1, fn="lbm_setup_static") == P.LBM_EWORKSPACE
    assert f"need {need} bytes".encode() in P.lib().lbm_last_error()
    assert _setup_rc(m, ws=fake, nbytes=need, fn="lbm_setup") == P.LBM_EWORKSPACE


def test_gather_span_bounds_brute_force(tmp_path):
    """The step kernels address a chunk's gathers from one base pointer with
    32-bit offsets; the host bound on how far they reach (gather_span) must
    cover every access, checked element by element on random images."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, "paper_1902_11193_amd", "csrc")
    exe = tmp_path / "check_span"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", csrc, os.path.join(root, "tests", "host", "check_span.cpp"),
                    os.path.join(csrc, "lbm_host.cpp"), "-o", str(exe), "-lpthread"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout


def test_bitmap_entries_decode_to_neighbour_table(tmp_path):
    """The bitmap index (packed coordinate per node; per row word and plane, a
    16-byte entry with rows y - 1, y, y + 1, plus the x- and y-wrap slots)
    decodes, by the step kernel's arithmetic modelled on the CPU, to exactly
    the pull sources of the neighbour table on random periodic and mirrored
    images, with every load in bounds, including row lengths around the
    18-voxel word step."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, "paper_1902_11193_amd", "csrc")
    exe = tmp_path / "check_bitmap"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", csrc, os.path.join(root, "tests", "host", "check_bitmap.cpp"),
                    os.path.join(csrc, "lbm_host.cpp"), "-o", str(exe), "-lpthread"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout


@pytest.mark.parametrize("shape,pad,my,mz", [((3, 4, 5), 2, True, True), ((4, 3, 6), 5, False, True),
                                             ((2, 5, 3), 0, True, False), ((3, 3, 3), 1, False, False)])
def test_boundary_image_pads_and_mirrors(shape, pad, my, mz):
    """Padding along x with fluid layers and reflection across the y / z faces
    (symmetry planes), checked against numpy."""
    m = random_mask(shape, 0.4, 7)
    want = m
    if my:
        want = np.concatenate([want, want[:, ::-1]], axis=1)
    if mz:
        want = np.concatenate([want, want[::-1]], axis=0)
    want = np.pad(want, ((0, 0), (0, 0), (pad, pad)))
    assert np.array_equal(P.lbm_boundary_image(m, pad, my, mz), want)


def test_boundary_image_rejects_bad_arguments():
    m = random_mask((3, 3, 3), 0.4, 7)
    with pytest.raises(P.LbmError) as e:
        P.lbm_boundary_image(m, -1)
    assert e.value.code == P.LBM_EINVAL


@pytest.mark.parametrize("shape", [(5, 6, 7), (40, 3, 9), (3, 2, 130)])
def test_neighbor_nodes_equal_the_full_table(shape):
    m = random_mask(shape, 0.3, 4)
    t = P.lbm_neighbor_table(m)
    rng = np.random.default_rng(1)
    pick = rng.choice(t.shape[1], min(50, t.shape[1]), replace=False)
    assert np.array_equal(P.lbm_neighbor_nodes(m, pick), t[:, pick])
    with pytest.raises(P.LbmError):
        P.lbm_neighbor_nodes(m, np.array([t.shape[1]]))
