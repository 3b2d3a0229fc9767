"""Python binding of liblbm, the MI355X D3Q19 MRT permeability solver.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides the device workspace and the stream.  The
functions with ``lbm_`` names map one-to-one onto the C-ABI in
``include/lbm.h``; ``Solver`` and ``permeability`` are conveniences over them.

The shared library must be built first (``python -m paper_1902_11193_amd.build``);
nothing here falls back to another implementation when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint8, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOFLUID, LBM_EWORKSPACE, LBM_EHIP, LBM_ENAN, LBM_ERANGE = 0, -1, -2, -3, -4, -5, -6
LBM_EBUSY = -7
LBM_REDUCTION_BYTES = 557312    # include/lbm.h
SETS = {"SRT": 0, "A": 1, "B": 2, "C": 3, "D": 4, "E": 5}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2, "f16r": 3}
INDEX = {"table": 0, "bitmap": 1}
COLLISION = {"mrt": 0, "trt": 1}
WALL = {"halfway": 0, "fullway": 1}

# Every symbol of include/lbm.h with its C signature.
SIGNATURES = {
    "lbm_velocities": (c_int, [POINTER(c_int)]),
    "lbm_rates": (c_int, [c_int, c_double, c_double, POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    "lbm_workspace_query": (c_int, [POINTER(c_uint8), c_int, c_int, c_int, c_int, c_int, POINTER(c_size_t),
                                    POINTER(c_int64)]),
    "lbm_neighbor_table": (c_int, [POINTER(c_uint8), c_int, c_int, c_int, POINTER(c_int32), c_int64]),
    "lbm_node_order": (c_int, [POINTER(c_uint8), c_int, c_int, c_int, POINTER(c_int64), c_int64]),
    "lbm_setup": (c_int, [POINTER(c_void_p), POINTER(c_uint8), c_int, c_int, c_int, c_double, c_double, c_int,
                          POINTER(c_double), c_int, c_int, c_void_p, c_size_t, c_void_p]),
    "lbm_setup_static": (c_int, [POINTER(c_void_p), POINTER(c_uint8), c_int, c_int, c_int, c_double, c_double,
                                 c_int, POINTER(c_double), c_int, c_int, c_void_p, c_size_t, c_void_p]),
    "lbm_step": (c_int, [c_void_p, c_int]),
    "lbm_steps_done": (c_int64, [c_void_p]),
    "lbm_mean_velocity": (c_int, [c_void_p, POINTER(c_double)]),
    "lbm_permeability": (c_int, [c_void_p, POINTER(c_double)]),
    "lbm_mass_deviation": (c_int, [c_void_p, POINTER(c_double)]),
    "lbm_mass": (c_int, [c_void_p, POINTER(c_double)]),
    "lbm_history": (c_int, [c_void_p, c_int, POINTER(c_double)]),
    "lbm_run_to_steady": (c_int, [c_void_p, c_double, c_int, c_int, POINTER(c_int), POINTER(c_double), POINTER(c_int)]),
    "lbm_get_state": (c_int, [c_void_p, POINTER(c_double)]),
    "lbm_set_state": (c_int, [c_void_p, POINTER(c_double)]),
    "lbm_fluid_index": (c_int, [c_void_p, POINTER(c_int64)]),
    "lbm_set_force_field": (c_int, [c_void_p, c_void_p]),
    "lbm_n_fluid": (c_int64, [c_void_p]),
    "lbm_set_storage_exponent": (c_int, [c_void_p, c_int]),
    "lbm_set_collision": (c_int, [c_void_p, c_int]),
    "lbm_wall_workspace_query": (c_int, [c_void_p, c_void_p]),
    "lbm_set_wall": (c_int, [c_void_p, c_int, c_void_p, c_size_t]),
    "lbm_set_pressure": (c_int, [c_void_p, c_int, c_double, c_double]),
    "lbm_neighbor_nodes": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_int64, c_void_p]),
    "lbm_get_state_nodes": (c_int, [c_void_p, c_void_p, c_int64, c_void_p]),
    "lbm_set_graphs": (c_int, [c_void_p, c_int]),
    "lbm_set_symmetry": (c_int, [c_void_p, c_int, c_int]),
    "lbm_boundary_dims": (c_int, [c_int, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "lbm_boundary_image": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_int, c_void_p]),
    "lbm_adjoint_workspace_query": (c_int, [c_void_p, c_int, c_int, POINTER(c_size_t)]),
    "lbm_adjoint": (c_int, [c_void_p, c_int, c_int, c_void_p, c_size_t, POINTER(c_double), POINTER(c_double),
                            POINTER(c_double), c_void_p]),
    "lbm_adjoint_timing": (c_int, [c_void_p, POINTER(c_double)]),
    "lbm_destroy": (None, [c_void_p]),
    "lbm_last_error": (ctypes.c_char_p, []),
}

_lib = None


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """The loaded liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1902_11193_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_last_error().decode())


def _geom(geometry: np.ndarray):
    g = np.ascontiguousarray(geometry, dtype=np.uint8)
    if g.ndim != 3:
        raise ValueError("geometry must be a 3-D uint8 array [nz][ny][nx]")
    nz, ny, nx = g.shape
    return g, nx, ny, nz


def _dptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(POINTER(ctype))


# ---------------------------------------------------------------- C-ABI mirrors
def lbm_velocities() -> np.ndarray:
    c = np.zeros((19, 3), np.int32)
    _check(lib().lbm_velocities(_dptr(c, c_int)))
    return c


def lbm_rates(relaxation_set, tau: float, Lambda: float = 0.0):
    s, dt, dl = (np.zeros(19) for _ in range(3))
    rs = SETS[relaxation_set] if isinstance(relaxation_set, str) else int(relaxation_set)
    _check(lib().lbm_rates(rs, float(tau), float(Lambda), _dptr(s, c_double), _dptr(dt, c_double),
                           _dptr(dl, c_double)))
    return s, dt, dl


def lbm_workspace_query(geometry, storage="f32", index="bitmap"):
    g, nx, ny, nz = _geom(geometry)
    nbytes, nf = c_size_t(0), c_int64(0)
    _check(lib().lbm_workspace_query(_dptr(g, c_uint8), nx, ny, nz, STORAGE[storage], INDEX[index],
                                     byref(nbytes), byref(nf)))
    return int(nbytes.value), int(nf.value)


def lbm_neighbor_table(geometry) -> np.ndarray:
    g, nx, ny, nz = _geom(geometry)
    nf = int(np.count_nonzero(g == 0))
    t = np.empty((18, max(nf, 1)), np.int32)
    _check(lib().lbm_neighbor_table(_dptr(g, c_uint8), nx, ny, nz, _dptr(t, c_int32), nf))
    return t[:, :nf]


def lbm_node_order(geometry) -> np.ndarray:
    """Linear voxel id of every node of the compacted fluid list (node order)."""
    g, nx, ny, nz = _geom(geometry)
    nf = int(np.count_nonzero(g == 0))
    v = np.empty(max(nf, 1), np.int64)
    _check(lib().lbm_node_order(_dptr(g, c_uint8), nx, ny, nz, _dptr(v, c_int64), nf))
    return v[:nf]


def lbm_neighbor_nodes(geometry, nodes) -> np.ndarray:
    """Pull sources (18, len(nodes)) of the given nodes (-1: solid source)."""
    g, nx, ny, nz = _geom(geometry)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    t = np.empty((18, max(len(nodes), 1)), np.int32)
    _check(lib().lbm_neighbor_nodes(_dptr(g, c_uint8), nx, ny, nz, _dptr(nodes, c_int64), len(nodes),
                                    _dptr(t, c_int32)))
    return t[:, :len(nodes)]


def lbm_boundary_image(geometry, pad: int = 5, mirror_y: bool = True, mirror_z: bool = True) -> np.ndarray:
    """The image padded along x with `pad` fluid layers per side and reflected
    across its y / z faces (symmetry planes in the periodic box)."""
    g, nx, ny, nz = _geom(geometry)
    o = (c_int * 3)()
    _check(lib().lbm_boundary_dims(nx, ny, nz, int(pad), int(bool(mirror_y)), int(bool(mirror_z)),
                                   ctypes.byref(o, 0), ctypes.byref(o, 4), ctypes.byref(o, 8)))
    out = np.empty((o[2], o[1], o[0]), np.uint8)
    _check(lib().lbm_boundary_image(_dptr(g, c_uint8), nx, ny, nz, int(pad), int(bool(mirror_y)),
                                    int(bool(mirror_z)), _dptr(out, c_uint8)))
    return out


def raster_permutation(geometry) -> np.ndarray:
    """perm with raster_list[perm[k]] = node k: position of every node in the
    raster-ordered (x fastest) list of fluid voxels."""
    g = np.ascontiguousarray(geometry, dtype=np.uint8)
    order = lbm_node_order(g)
    raster = np.flatnonzero(g.reshape(-1) == 0)
    return np.searchsorted(raster, order)


# ---------------------------------------------------------------- solver
class Solver:
    """One voxel image on one GPU: owns the library context and its workspace."""

    def __init__(self, geometry, tau: float, Lambda: float | None = None, relaxation_set="E",
                 g=(1e-6, 0.0, 0.0), storage="f32", index="bitmap", device="cuda", static_scratch=False):
        """static_scratch: set up with lbm_setup_static (the reduction scratch in
        the library's static array; the workspace is LBM_REDUCTION_BYTES smaller)."""
        import torch

        self._torch = torch
        gm, nx, ny, nz = _geom(geometry)
        self.shape = gm.shape
        self.tau, self.Lambda, self.g = float(tau), (None if Lambda is None else float(Lambda)), tuple(map(float, g))
        self.storage, self.index = storage, index
        self.relaxation_set = relaxation_set
        nbytes, self.n_fluid = lbm_workspace_query(gm, storage, index)
        if static_scratch:
            nbytes -= LBM_REDUCTION_BYTES
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        ctx = c_void_p()
        gv = (c_double * 3)(*self.g)
        rs = SETS[relaxation_set] if isinstance(relaxation_set, str) else int(relaxation_set)
        setup = lib().lbm_setup_static if static_scratch else lib().lbm_setup
        _check(setup(byref(ctx), _dptr(gm, c_uint8), nx, ny, nz, self.tau,
                     0.0 if Lambda is None else float(Lambda), rs, gv, STORAGE[storage],
                     INDEX[index], c_void_p(self.workspace.data_ptr()), nbytes,
                     c_void_p(self.stream.cuda_stream)))
        self._ctx = ctx
        self._field = None
        self._wall_ws = None

    # -- stepping and observables
    def step(self, n: int = 1):
        _check(lib().lbm_step(self._ctx, int(n)))

    @property
    def steps_done(self) -> int:
        return int(lib().lbm_steps_done(self._ctx))

    def mean_velocity(self) -> np.ndarray:
        u = np.zeros(3)
        _check(lib().lbm_mean_velocity(self._ctx, _dptr(u, c_double)))
        return u

    def permeability(self) -> np.ndarray:
        k = np.zeros(3)
        _check(lib().lbm_permeability(self._ctx, _dptr(k, c_double)))
        return k

    def mass(self) -> float:
        """Total mass sum_fluid rho at the last step."""
        d = c_double()
        _check(lib().lbm_mass(self._ctx, byref(d)))
        return d.value

    def mass_deviation(self) -> float:
        d = c_double(0)
        _check(lib().lbm_mass_deviation(self._ctx, byref(d)))
        return d.value

    def history(self, count: int) -> np.ndarray:
        u = np.zeros((count, 3))
        _check(lib().lbm_history(self._ctx, int(count), _dptr(u, c_double)))
        return u

    def run_to_steady(self, eps=1e-6, check_every=100, max_steps=100000):
        steps, conv = c_int(0), c_int(0)
        k = np.zeros(3)
        _check(lib().lbm_run_to_steady(self._ctx, float(eps), int(check_every), int(max_steps),
                                       byref(steps), _dptr(k, c_double), byref(conv)))
        return dict(steps=steps.value, k=k, converged=bool(conv.value))

    # -- state
    def get_state(self) -> np.ndarray:
        f = np.zeros((19, self.n_fluid))
        _check(lib().lbm_get_state(self._ctx, _dptr(f, c_double)))
        return f

    def get_state_nodes(self, nodes) -> np.ndarray:
        """Full populations (19, len(nodes)) of the given nodes only."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        f = np.zeros((19, max(len(nodes), 1)))
        _check(lib().lbm_get_state_nodes(self._ctx, _dptr(nodes, c_int64), len(nodes), _dptr(f, c_double)))
        return f[:, :len(nodes)]

    def set_state(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (19, self.n_fluid):
            raise ValueError("state must be (19, n_fluid)")
        _check(lib().lbm_set_state(self._ctx, _dptr(f, c_double)))

    def fluid_index(self) -> np.ndarray:
        v = np.zeros(self.n_fluid, np.int64)
        _check(lib().lbm_fluid_index(self._ctx, _dptr(v, c_int64)))
        return v

    def set_force_field(self, g_field):
        """Per-node accelerations, a CUDA float32 tensor (3, n_fluid); None = uniform g."""
        if g_field is None:
            self._field = None
            _check(lib().lbm_set_force_field(self._ctx, None))
            return
        t = self._torch
        if g_field.device.type != "cuda" or g_field.dtype != t.float32 or tuple(g_field.shape) != (3, self.n_fluid):
            raise ValueError("g_field must be a CUDA float32 tensor of shape (3, n_fluid)")
        self._field = g_field.contiguous()
        _check(lib().lbm_set_force_field(self._ctx, c_void_p(self._field.data_ptr())))

    def set_storage_exponent(self, e: int):
        _check(lib().lbm_set_storage_exponent(self._ctx, int(e)))

    def set_graphs(self, enable: bool):
        """Replay captured 32-step graphs (default) or launch every step."""
        _check(lib().lbm_set_graphs(self._ctx, int(bool(enable))))

    def set_collision(self, kind: str):
        """'mrt' (moment space, any set) or 'trt' (link-wise, SRT / B / E)."""
        _check(lib().lbm_set_collision(self._ctx, COLLISION[kind]))

    def set_pressure(self, rho_in: float | None, rho_out: float | None = None):
        """Zou-He pressure faces at x = 0 / nx - 1 with these densities; None: periodic again."""
        if rho_in is None:
            _check(lib().lbm_set_pressure(self._ctx, 0, 1.0, 1.0))
        else:
            _check(lib().lbm_set_pressure(self._ctx, 1, float(rho_in), float(rho_out)))

    def set_symmetry(self, mirror_y: bool, mirror_z: bool):
        """Symmetry (mirror) planes on the y and/or z faces (bitmap index, FP32)."""
        _check(lib().lbm_set_symmetry(self._ctx, int(bool(mirror_y)), int(bool(mirror_z))))

    def set_wall(self, kind: str):
        """'halfway' (default) or 'fullway' bounce-back (FP32 storage)."""
        if kind == "halfway":
            _check(lib().lbm_set_wall(self._ctx, WALL[kind], None, 0))
            self._wall_ws = None
            return
        nbytes = c_size_t(0)
        _check(lib().lbm_wall_workspace_query(self._ctx, byref(nbytes)))
        ws = self._torch.empty(nbytes.value, dtype=self._torch.uint8, device=self.device)
        _check(lib().lbm_set_wall(self._ctx, WALL[kind], c_void_p(ws.data_ptr()), nbytes.value))
        self._wall_ws = ws

    # -- adjoint
    def adjoint(self, n_steps: int, checkpoint_every: int = 200):
        """k_N and dk/dtau, dk/dLambda, dk/dg (CUDA float64 (3, n_fluid))."""
        t = self._torch
        nb = c_size_t(0)
        _check(lib().lbm_adjoint_workspace_query(self._ctx, int(n_steps), int(checkpoint_every), byref(nb)))
        ws = t.empty(int(nb.value), dtype=t.uint8, device=self.device)
        dg = t.empty((3, self.n_fluid), dtype=t.float64, device=self.device)
        k, dt, dl = c_double(0), c_double(0), c_double(0)
        _check(lib().lbm_adjoint(self._ctx, int(n_steps), int(checkpoint_every), c_void_p(ws.data_ptr()),
                                 nb.value, byref(k), byref(dt), byref(dl), c_void_p(dg.data_ptr())))
        del ws
        return dict(k=k.value, dk_dtau=dt.value, dk_dLambda=dl.value, dk_dg=dg)

    def adjoint_timing(self) -> dict:
        """GPU milliseconds of the last adjoint: forward, recompute, reverse."""
        ms = np.zeros(3)
        _check(lib().lbm_adjoint_timing(self._ctx, _dptr(ms, c_double)))
        return dict(forward_ms=ms[0], recompute_ms=ms[1], reverse_ms=ms[2])

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().lbm_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_fn():
    import torch

    class PermeabilityFn(torch.autograd.Function):
        """k_N(tau, Lambda, g(x)) with gradients from the library's discrete adjoint."""

        @staticmethod
        def forward(ctx, tau, Lambda, g_field, geometry, relaxation_set, g_ref, n_steps, checkpoint_every, index):
            s = Solver(geometry, float(tau), float(Lambda), relaxation_set, g_ref, "f32", index,
                       device=g_field.device)
            s.set_force_field(g_field.detach().float().contiguous())
            s.step(n_steps)
            axis = int(np.argmax(np.abs(np.asarray(g_ref))))
            k = float(s.permeability()[axis])
            ctx.solver = s
            ctx.meta = (n_steps, checkpoint_every)
            return torch.tensor(k, dtype=torch.float64, device=g_field.device)

        @staticmethod
        def backward(ctx, gk):
            n_steps, K = ctx.meta
            r = ctx.solver.adjoint(n_steps, K)
            ctx.solver.close()
            dev = gk.device
            gt = gk * torch.tensor(r["dk_dtau"], dtype=torch.float64, device=dev)
            gl = gk * torch.tensor(r["dk_dLambda"], dtype=torch.float64, device=dev)
            gg = (gk * r["dk_dg"]).to(torch.float32)
            return gt, gl, gg, None, None, None, None, None, None

    return PermeabilityFn


def permeability(geometry, tau, Lambda, g_field, relaxation_set="E", g_ref=(1e-6, 0.0, 0.0),
                 n_steps=1000, checkpoint_every=200, index="bitmap"):
    """Differentiable k_N: ``tau`` and ``Lambda`` are 0-d tensors, ``g_field`` a
    CUDA tensor (3, n_fluid) of per-node accelerations (normally g_ref everywhere)."""
    return _autograd_fn().apply(tau, Lambda, g_field, geometry, relaxation_set, tuple(g_ref), int(n_steps),
                                int(checkpoint_every), index)


__all__ = ["lib", "LbmError", "Solver", "permeability", "lbm_velocities", "lbm_rates", "lbm_workspace_query",
           "lbm_neighbor_table", "lbm_neighbor_nodes", "lbm_node_order", "lbm_boundary_image", "raster_permutation", "SIGNATURES", "SETS", "STORAGE", "INDEX", "COLLISION", "WALL", "LIB_PATH"]
