"""ctypes binding of the C ABI in include/lbm.h (liblbm13.so).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch provides the device arena (a uint8 tensor) and the
stream.  The library must have been built (``__graft_entry__.build()`` or
``python paper_1910_13515_amd/build.py``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm13.so")

LBM_OK = 0
LBM_E_INVAL = -1
LBM_E_NOMEM = -2
LBM_E_DEVICE = -3
LBM_E_NONREALIZABLE = -4
LBM_E_NEWTON = -5
LBM_E_NONFINITE = -6

STATUS_NAMES = {0: "LBM_OK", -1: "LBM_E_INVAL", -2: "LBM_E_NOMEM", -3: "LBM_E_DEVICE", -4: "LBM_E_NONREALIZABLE",
                -5: "LBM_E_NEWTON", -6: "LBM_E_NONFINITE"}

LBM_STORE_FP64 = 0
LBM_STORE_FP32_SHIFTED = 1
LBM_STORE_FP16_SHIFTED = 2
STORAGE = {"fp64": LBM_STORE_FP64, "fp32s": LBM_STORE_FP32_SHIFTED, "fp16s": LBM_STORE_FP16_SHIFTED}

LBM_FACE_PERIODIC = 0
LBM_FACE_EQUILIBRIUM = 1
LBM_FACE_NEUMANN = 2

EXPORTED = ["lbm_version", "lbm_velocities", "lbm_required_bytes", "lbm_create", "lbm_step", "lbm_moments",
            "lbm_moments_noalloc", "lbm_diagnostics",
            "lbm_get_state", "lbm_set_state", "lbm_get_info", "lbm_destroy", "lbm_last_error",
            "lbm_pool_overhead_bytes", "lbm_pool_create", "lbm_pool_admit", "lbm_pool_launch", "lbm_pool_wait",
            "lbm_pool_run", "lbm_pool_slot_progress", "lbm_pool_moments", "lbm_pool_release", "lbm_pool_get_info",
            "lbm_pool_destroy", "lbm_pool_last_error"]


# root finders of the multipliers: Newton-Raphson, or the secant variant
ROOT_FINDER = {"newton": 0, "secant": 1}


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("shift_ref", ctypes.c_int32), ("kn_relax", ctypes.c_int32),
        ("newton_maxit", ctypes.c_int32), ("faces", ctypes.c_int32 * 6),
        ("gamma", ctypes.c_double), ("mach", ctypes.c_double), ("reynolds", ctypes.c_double),
        ("length_ref", ctypes.c_double), ("rho_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("u_dir", ctypes.c_double * 3), ("tau", ctypes.c_double), ("newton_tol", ctypes.c_double),
        ("solid", ctypes.c_void_p), ("init_rho", ctypes.c_void_p), ("init_u", ctypes.c_void_p),
        ("init_T", ctypes.c_void_p), ("root_finder", ctypes.c_int32),
    ]


class lbm_step_stats(ctypes.Structure):
    _fields_ = [
        ("cell_updates", ctypes.c_int64), ("iterations", ctypes.c_int64), ("max_iterations", ctypes.c_int64),
        ("failed", ctypes.c_int64), ("cold_restarts", ctypes.c_int64), ("alpha_hist", ctypes.c_int64 * 4),
        ("wave_iterations", ctypes.c_int64), ("waves", ctypes.c_int64),
    ]


class lbm_info(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double), ("u_ref", ctypes.c_double * 3), ("shear_response", ctypes.c_double),
        ("delta", ctypes.c_double), ("cells", ctypes.c_int64), ("fluid_cells", ctypes.c_int64),
        ("steps_done", ctypes.c_int64), ("arena_bytes_used", ctypes.c_int64),
    ]


LBM_SCHED_ALL = 0
LBM_SCHED_SRPT = 1
LBM_SCHED_VFT = 2
SCHED = {"all": LBM_SCHED_ALL, "srpt": LBM_SCHED_SRPT, "vft": LBM_SCHED_VFT}


class lbm_pool_info(ctypes.Structure):
    _fields_ = [
        ("max_slots", ctypes.c_int32), ("active", ctypes.c_int32), ("running", ctypes.c_int32),
        ("graph_steps", ctypes.c_int32), ("sched", ctypes.c_int32), ("in_flight", ctypes.c_int32),
        ("fill_cells", ctypes.c_int64), ("arena_bytes", ctypes.c_int64), ("free_bytes", ctypes.c_int64),
        ("largest_free", ctypes.c_int64),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load liblbm13.so.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch first: the library's HIP runtime dependency must resolve to the
    # runtime torch has loaded, which owns the device arenas handed to it (a
    # second HIP runtime in the process does not see the device)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.lbm_version.restype = i32
    L.lbm_velocities.restype = ctypes.c_int
    L.lbm_velocities.argtypes = [vp]
    L.lbm_required_bytes.restype = i64
    L.lbm_required_bytes.argtypes = [ctypes.POINTER(lbm_params)]
    L.lbm_create.restype = ctypes.c_int
    L.lbm_create.argtypes = [ctypes.POINTER(lbm_params), vp, i64, vp, ctypes.POINTER(vp)]
    L.lbm_step.restype = ctypes.c_int
    L.lbm_step.argtypes = [vp, i32, ctypes.POINTER(lbm_step_stats)]
    L.lbm_moments.restype = ctypes.c_int
    L.lbm_moments.argtypes = [vp, vp, vp]
    L.lbm_moments_noalloc.restype = ctypes.c_int
    L.lbm_moments_noalloc.argtypes = [vp, vp, vp]
    L.lbm_diagnostics.restype = ctypes.c_int
    L.lbm_diagnostics.argtypes = [vp, vp, vp]
    L.lbm_get_state.restype = ctypes.c_int
    L.lbm_get_state.argtypes = [vp, vp, vp, vp]
    L.lbm_set_state.restype = ctypes.c_int
    L.lbm_set_state.argtypes = [vp, vp, vp, vp]
    L.lbm_get_info.restype = ctypes.c_int
    L.lbm_get_info.argtypes = [vp, ctypes.POINTER(lbm_info)]
    L.lbm_destroy.restype = ctypes.c_int
    L.lbm_destroy.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_last_error.argtypes = [vp]
    L.lbm_pool_overhead_bytes.restype = i64
    L.lbm_pool_overhead_bytes.argtypes = [i32]
    L.lbm_pool_create.restype = ctypes.c_int
    L.lbm_pool_create.argtypes = [i32, i32, i32, i32, i64, vp, i64, vp, ctypes.POINTER(vp)]
    L.lbm_pool_admit.restype = ctypes.c_int
    L.lbm_pool_admit.argtypes = [vp, ctypes.POINTER(lbm_params), i32, ctypes.POINTER(i32)]
    L.lbm_pool_launch.restype = ctypes.c_int
    L.lbm_pool_launch.argtypes = [vp, ctypes.POINTER(i32)]
    L.lbm_pool_wait.restype = ctypes.c_int
    L.lbm_pool_wait.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.lbm_pool_run.restype = ctypes.c_int
    L.lbm_pool_run.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.lbm_pool_slot_progress.restype = ctypes.c_int
    L.lbm_pool_slot_progress.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.lbm_pool_moments.restype = ctypes.c_int
    L.lbm_pool_moments.argtypes = [vp, i32, vp, vp]
    L.lbm_pool_release.restype = ctypes.c_int
    L.lbm_pool_release.argtypes = [vp, i32]
    L.lbm_pool_get_info.restype = ctypes.c_int
    L.lbm_pool_get_info.argtypes = [vp, ctypes.POINTER(lbm_pool_info)]
    L.lbm_pool_destroy.restype = ctypes.c_int
    L.lbm_pool_destroy.argtypes = [vp]
    L.lbm_pool_last_error.restype = ctypes.c_char_p
    L.lbm_pool_last_error.argtypes = [vp]
    _lib = L
    return L


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, ctx=None) -> int:
    if code < 0:
        raise LbmError(code, load().lbm_last_error(ctx).decode())
    return code


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# thin wrappers with the C names -------------------------------------------

def lbm_version() -> int:
    return load().lbm_version()


def lbm_velocities() -> np.ndarray:
    out = np.zeros(39 * 3, dtype=np.int32)
    _check(load().lbm_velocities(_ptr(out)))
    return out.reshape(39, 3)


def lbm_required_bytes(params: lbm_params) -> int:
    return _check(load().lbm_required_bytes(ctypes.byref(params)))


def lbm_create(params: lbm_params, arena_ptr: int, arena_bytes: int, stream_ptr: int):
    ctx = ctypes.c_void_p()
    _check(load().lbm_create(ctypes.byref(params), ctypes.c_void_p(arena_ptr), arena_bytes,
                             ctypes.c_void_p(stream_ptr), ctypes.byref(ctx)))
    return ctx


def lbm_step(ctx, nsteps: int, with_stats: bool = False):
    st = lbm_step_stats() if with_stats else None
    code = load().lbm_step(ctx, int(nsteps), ctypes.byref(st) if st is not None else None)
    if code == LBM_E_NEWTON and st is not None:
        return st, code
    _check(code, ctx)
    return st, code


def lbm_moments(ctx, n: int, fields: bool = True):
    out = np.empty(5 * n) if fields else None
    tot = np.empty(5)
    code = load().lbm_moments(ctx, _ptr(out), _ptr(tot))
    if code != LBM_E_NONFINITE:
        _check(code, ctx)
    return (None if out is None else out.reshape(5, n)), tot, code


def lbm_moments_noalloc(ctx, dev_out_ptr: int):
    """Totals (5 doubles) of the current state; the 5*N per-cell fields go to
    the caller's device buffer at dev_out_ptr (e.g. a torch float64 tensor's
    data_ptr()).  No device allocation anywhere in the call."""
    tot = np.empty(5)
    code = load().lbm_moments_noalloc(ctx, ctypes.c_void_p(dev_out_ptr), _ptr(tot))
    if code != LBM_E_NONFINITE:
        _check(code, ctx)
    return tot, code


def lbm_diagnostics(ctx, n: int):
    """(eps[N], iterations[N]) of the next step from the current state."""
    eps = np.empty(n)
    its = np.empty(n, dtype=np.int32)
    _check(load().lbm_diagnostics(ctx, _ptr(eps), _ptr(its)), ctx)
    return eps, its


def lbm_get_state(ctx, n: int):
    f = np.empty(39 * n)
    g = np.empty(39 * n)
    lam = np.empty(13 * n)
    _check(load().lbm_get_state(ctx, _ptr(f), _ptr(g), _ptr(lam)), ctx)
    return f, g, lam


def lbm_set_state(ctx, f, g, lam, n: int):
    """f, g: 39*n doubles each, lam: 13*n (the library reads exactly that many)."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
    lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
    if f.size != 39 * n or g.size != 39 * n or lam.size != 13 * n:
        raise ValueError(f"state of {n} cells needs 39n, 39n and 13n values; got {f.size}, {g.size}, {lam.size}")
    _check(load().lbm_set_state(ctx, _ptr(f), _ptr(g), _ptr(lam)), ctx)


def lbm_get_info(ctx) -> lbm_info:
    info = lbm_info()
    _check(load().lbm_get_info(ctx, ctypes.byref(info)), ctx)
    return info


def lbm_destroy(ctx):
    _check(load().lbm_destroy(ctx))


def make_params(shape, storage="fp64", gamma=1.4, mach=0.0, reynolds=0.0, length_ref=0.0, rho_ref=1.0, T_ref=0.5,
                u_dir=(1.0, 0.0, 0.0), tau=0.0, kn_relax=True, faces=(0,) * 6, newton_tol=0.0, newton_maxit=0,
                shift_ref=0, root_finder=0):
    p = lbm_params()
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.shift_ref = int(shift_ref)
    p.kn_relax = int(bool(kn_relax))
    p.newton_maxit = int(newton_maxit)
    for k in range(6):
        p.faces[k] = int(faces[k])
    p.gamma = float(gamma)
    p.mach = float(mach)
    p.reynolds = float(reynolds)
    p.length_ref = float(length_ref)
    p.rho_ref = float(rho_ref)
    p.T_ref = float(T_ref)
    for k in range(3):
        p.u_dir[k] = float(u_dir[k])
    p.tau = float(tau)
    p.newton_tol = float(newton_tol)
    p.root_finder = ROOT_FINDER[root_finder] if isinstance(root_finder, str) else int(root_finder)
    return p


class Solver:
    """One solve on the current GPU: owns a torch uint8 arena and an lbm_ctx.

    ``fields`` = (rho[N], u[3, N], T[N]) float64 arrays or None (reference
    state); ``solid`` = uint8 array of N or None."""

    def __init__(self, shape, fields=None, solid=None, stream=None, **kw):
        import torch
        load()
        self.shape = tuple(int(v) for v in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.params = make_params(self.shape, **kw)
        self._keep = []
        if solid is not None:
            s = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
            if s.size != self.n:
                raise ValueError(f"solid mask has {s.size} cells, the grid {self.n}")
            self._keep.append(s)
            self.params.solid = s.ctypes.data
        if fields is not None:
            rho, u, T = (np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in fields)
            if rho.size != self.n or u.size != 3 * self.n or T.size != self.n:
                raise ValueError(f"fields of {self.n} cells need n, 3n and n values; got {rho.size}, {u.size}, {T.size}")
            self._keep += [rho, u, T]
            self.params.init_rho = rho.ctypes.data
            self.params.init_u = u.ctypes.data
            self.params.init_T = T.ctypes.data
        self.bytes = lbm_required_bytes(self.params)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.arena = torch.empty(self.bytes + 256, dtype=torch.uint8, device="cuda")
        base = self.arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.ctx = lbm_create(self.params, aligned, self.bytes, self.stream.cuda_stream)
        self._keep = []  # host inputs are copied during create

    @classmethod
    def from_params(cls, params: lbm_params, stream=None):
        """A solve from ready lbm_params (host inputs it points to must stay
        alive for this call only: the library copies them during create)."""
        import torch
        load()
        s = cls.__new__(cls)
        s.shape = (int(params.nx), int(params.ny), int(params.nz))
        s.n = s.shape[0] * s.shape[1] * s.shape[2]
        s.params = params
        s._keep = []
        s.bytes = lbm_required_bytes(params)
        s.stream = stream if stream is not None else torch.cuda.current_stream()
        s.arena = torch.empty(s.bytes + 256, dtype=torch.uint8, device="cuda")
        aligned = (s.arena.data_ptr() + 255) // 256 * 256
        s.ctx = lbm_create(params, aligned, s.bytes, s.stream.cuda_stream)
        return s

    def step(self, nsteps=1, stats=False):
        st, code = lbm_step(self.ctx, nsteps, with_stats=stats)
        return st

    def moments(self, fields=True):
        out, tot, code = lbm_moments(self.ctx, self.n, fields)
        return out, tot

    def get_state(self):
        return lbm_get_state(self.ctx, self.n)

    def diagnostics(self):
        """Knudsen sensor and Newton iterations of the next step, per cell."""
        return lbm_diagnostics(self.ctx, self.n)

    def set_state(self, f, g, lam):
        lbm_set_state(self.ctx, f, g, lam, self.n)

    def info(self) -> lbm_info:
        return lbm_get_info(self.ctx)

    def close(self):
        if self.ctx is not None:
            lbm_destroy(self.ctx)
            self.ctx = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
