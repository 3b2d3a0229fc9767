"""Shared helpers of the GPU parity tests: run the library and the oracle on the
same seeded input and map between their velocity orders."""
import numpy as np
import torch

import oracle as O
import paper_1902_11193_amd as P

ORC_C = O.velocities().numpy()
LIB_C = P.lbm_velocities()
# oracle index k holds library population PERM[k]
PERM = np.array([int(np.flatnonzero((LIB_C == ORC_C[k]).all(1))[0]) for k in range(19)])
W_LIB = np.array([1 / 3 if not c.any() else (1 / 18 if abs(c).sum() == 1 else 1 / 36) for c in LIB_C])


def banner(msg: str):
    """Names the case on stdout before any GPU work starts."""
    print(f"[gpu-case] {msg}", flush=True)


def oracle_problem(mask, tau, Lam, rset, g, linear=False):
    return O.Problem(mask, tau, Lam, rset, g, linear=linear)


def _perm(problem):
    """Raster position (among fluid voxels) of every library node."""
    if not hasattr(problem, "_lib_perm"):
        problem._lib_perm = P.raster_permutation(problem.solid.numpy().astype(np.uint8))
    return problem._lib_perm


def dense_from_lib(problem, f_lib):
    """Library state (19, nf): library velocity and node order -> oracle dense (19, nz, ny, nx)."""
    raster = np.empty_like(f_lib)
    raster[:, _perm(problem)] = f_lib
    fh = torch.zeros((19,) + problem.shape, dtype=torch.float64)
    fh[:, problem.fluid] = torch.from_numpy(raster[PERM])
    return fh


def lib_from_dense(problem, fh):
    """Oracle dense state -> (19, nf) in library velocity and node order."""
    f_orc = fh[:, problem.fluid].numpy()
    out = np.empty_like(f_orc)
    out[PERM] = f_orc
    return out[:, _perm(problem)]


def nodes_from_raster(mask, a):
    """Per-fluid-voxel array (..., nf) in raster order -> library node order."""
    return a[..., P.raster_permutation(mask)]


def random_state(nf, seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    return W_LIB[:, None] + amp * rng.standard_normal((19, nf))


def deviation_error(a, b):
    """max |a - b| over populations, relative to max |b - w|."""
    scale = np.abs(b - W_LIB[:, None]).max()
    return np.abs(a - b).max() / scale
