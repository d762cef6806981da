"""FP64 CPU oracle for the D3Q39 13-moment DDF lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_1910_13515_amd``) never does, and the two share no code.

The arithmetic lives in ``lbm_oracle.c`` (plain C, FP64, optional OpenMP); this
module is ctypes marshalling plus the helpers the tests need: the exact Riemann
solver (``riemann.py``) and the relaxation time from the Reynolds number.

Parity status of each function (what pins it, see ``tests/test_oracle_*.py``):
  * orc_equilibrium: 13 Maxwell-Boltzmann moments from Gauss-Hermite quadrature
    of the continuous Maxwellian; u = 0 reduction to a 1-D root find;
    high-precision convex-dual solve (mpmath); cubic symmetry; rho scaling.
  * orc_step: brute force on 4^3 grids (explicit modular indexing, scipy/mpmath
    equilibrium); conservation of mass, momentum and energy; shear-wave decay
    against the Navier-Stokes rate; sound speed sqrt(gamma T); Sod shock tube
    against the exact Riemann solution; streaming permutation against numpy.roll.
  * orc_moments: the totals are checked against direct sums in the tests.
  * orc_equilibrium_secant / root_finder 1 (the secant variant): the shift
    matrix against the shifted basis at random points; the model Jacobian
    against Gauss-Hermite moments of the continuous Maxwellian; convergence
    to the same (unique) equilibrium as the 32-digit solve; its first update
    at rest equal to Newton's; a step equal to the Newton step within the
    stopping bound.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the same source built with fused multiply-add contraction: a second
# rounding of the same arithmetic, used to measure how fast round-off
# differences grow along a trajectory (the floor any other implementation
# can be compared against)
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")

NQ = 39
NL = 13

FACE_PERIODIC, FACE_EQUILIBRIUM, FACE_NEUMANN = 0, 1, 2
CELL_FLUID, CELL_SOLID, CELL_FROZEN, CELL_NEUMANN = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction), and the
    FMA-contracted variant."""
    for out, extra in ((LIB, ["-ffp-contract=off"]), (LIB_FMA, ["-mfma", "-mavx2", "-ffp-contract=fast"])):
        if force or not os.path.exists(out):
            cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp"] + extra + ["-o", out + ".tmp", SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(out + ".tmp", out)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("kn_relax", ctypes.c_int32), ("newton_maxit", ctypes.c_int32),
        ("faces", ctypes.c_int32 * 6),
        ("gamma", ctypes.c_double), ("tau", ctypes.c_double), ("newton_tol", ctypes.c_double),
        ("solid", ctypes.c_void_p),
        ("floor_rule", ctypes.c_int32), ("skip_cold_after_failure", ctypes.c_int32),
        ("root_finder", ctypes.c_int32), ("model_T", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int64), ("max_iterations", ctypes.c_int64),
        ("failed", ctypes.c_int64), ("alpha_hist", ctypes.c_int64 * 4),
        ("cold_restarts", ctypes.c_int64), ("evaluations", ctypes.c_int64),
    ]


_libs = {}


def lib(variant: str = "plain"):
    """The compiled oracle; variant "fma" is the FMA-contracted build."""
    if variant not in _libs:
        path = LIB if variant == "plain" else LIB_FMA
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_equilibrium.restype = ctypes.c_int
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_int, dp, dp]
        L.orc_equilibrium_secant.restype = ctypes.c_int
        L.orc_equilibrium_secant.argtypes = [ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp]
        L.orc_model_jacobian.restype = ctypes.c_int
        L.orc_model_jacobian.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_void_p, dp, dp]
        L.orc_init.restype = ctypes.c_int64
        L.orc_step.restype = None
        L.orc_moments.restype = None
        L.orc_stream_only.restype = None
        _libs[variant] = L
    return _libs[variant]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def velocities() -> np.ndarray:
    out = np.zeros(NQ * 3, dtype=np.int32)
    lib().orc_velocities(_ptr(out))
    return out.reshape(NQ, 3)


def equilibrium(rho, u, T, gamma=1.4, lam=None, tol=1e-13, maxit=100):
    """Equilibrium of one cell.  Returns (feq, geq, lam, iterations).

    Cold start (Maxwellian-shaped guess) when ``lam`` is None."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    cold = lam is None
    lam = np.zeros(NL) if cold else np.array(lam, dtype=np.float64)
    feq = np.zeros(NQ)
    geq = np.zeros(NQ)
    it = lib().orc_equilibrium(float(rho), _dptr(u), float(T), float(gamma), _dptr(lam), int(cold), float(tol),
                               int(maxit), _dptr(feq), _dptr(geq))
    return feq, geq, lam, it


def equilibrium_secant(rho, u, T, T_ref, gamma=1.4, lam=None, tol=1e-13, maxit=100):
    """Equilibrium of one cell by the secant variant (model Jacobian on the
    rest equilibrium at T_ref).  Returns (feq, geq, lam, iterations)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    cold = lam is None
    lam = np.zeros(NL) if cold else np.array(lam, dtype=np.float64)
    feq = np.zeros(NQ)
    geq = np.zeros(NQ)
    it = lib().orc_equilibrium_secant(float(rho), _dptr(u), float(T), float(T_ref), float(gamma), _dptr(lam),
                                      int(cold), float(tol), int(maxit), _dptr(feq), _dptr(geq))
    return feq, geq, lam, it


def model_jacobian(u, T, T_ref, J_rest=None):
    """(J_model, A(u)) of the secant variant; J_rest (13 x 13) replaces the
    lattice's rest Jacobian at T_ref when given."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    J = np.zeros((NL, NL))
    A = np.zeros((NL, NL))
    jr = None if J_rest is None else np.ascontiguousarray(J_rest, dtype=np.float64)
    rc = lib().orc_model_jacobian(_dptr(u), float(T), float(T_ref), None if jr is None else _ptr(jr), _dptr(J),
                                  _dptr(A))
    if rc != 0:
        raise RuntimeError("no rest equilibrium at this temperature")
    return J, A


def shear_response(T: float, du: float = 1e-4) -> float:
    """K(T) = d/du_y sum_i f^eq_i xi_x^2 xi_y at rest, per unit density, by a
    central difference of this oracle's equilibrium.  The BGK lattice step has
    shear viscosity nu = K (tau - 1/2); the continuous Maxwellian would give
    K = T, but the 13 constraints fix only the contracted third moment."""
    c = velocities().astype(np.float64)
    fp, _, _, _ = equilibrium(1.0, [0.0, du, 0.0], T, tol=1e-15)
    fm, _, _, _ = equilibrium(1.0, [0.0, -du, 0.0], T, tol=1e-15)
    return float(((fp - fm) * c[:, 0] ** 2 * c[:, 1]).sum() / (2.0 * du))


def tau_from_reynolds(speed: float, length: float, reynolds: float, T_ref: float) -> float:
    """Relaxation time for a Reynolds number.  Reading (the paper is silent):
    Re = |u| L / nu with the model's own shear viscosity nu = K(T_ref)
    (tau - 1/2), so tau = 1/2 + |u| L / (Re K)."""
    return 0.5 + speed * length / (reynolds * shear_response(T_ref))


class Oracle:
    """A grid, its parameters and its FP64 state (populations f, g and the
    multipliers lam, SoA ``[39][N]`` / ``[13][N]`` with x fastest)."""

    def __init__(self, nx, ny, nz, gamma=1.4, tau=0.6, kn_relax=True, faces=(0,) * 6, solid=None,
                 newton_tol=1e-13, newton_maxit=30, variant="plain", floor_rule=True,
                 skip_cold_after_failure=True, root_finder=0, model_T=0.5):
        self.L = lib(variant)
        self.shape = (nx, ny, nz)
        self.n = nx * ny * nz
        self.gamma = float(gamma)
        self.tau = float(tau)
        self.solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        if self.solid is not None and self.solid.size != self.n:
            raise ValueError("solid mask size does not match the grid")
        p = _Params()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.kn_relax = int(bool(kn_relax))
        p.newton_maxit = int(newton_maxit)
        for k in range(6):
            p.faces[k] = int(faces[k])
        p.gamma = self.gamma
        p.tau = self.tau
        p.newton_tol = float(newton_tol)
        p.solid = _ptr(self.solid) if self.solid is not None else None
        p.floor_rule = int(bool(floor_rule))
        p.skip_cold_after_failure = int(bool(skip_cold_after_failure))
        p.root_finder = int(root_finder)
        p.model_T = float(model_T)
        self.p = p
        self.f = np.zeros(NQ * self.n)
        self.g = np.zeros(NQ * self.n)
        self.lam = np.zeros(NL * self.n)
        self.stats = Stats()

    # fields are SoA numpy arrays of length N (u: 3N) in x-fastest order
    def init(self, rho, u, T) -> int:
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        assert rho.size == self.n and u.size == 3 * self.n and T.size == self.n
        return int(self.L.orc_init(ctypes.byref(self.p), _ptr(rho), _ptr(u), _ptr(T), _ptr(self.f), _ptr(self.g),
                                  _ptr(self.lam)))

    def set_state(self, f, g, lam):
        self.f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1).copy()
        self.g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1).copy()
        self.lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1).copy()
        assert self.f.size == NQ * self.n and self.g.size == NQ * self.n and self.lam.size == NL * self.n

    def step(self, nsteps=1, diagnostics=False):
        fo = np.empty_like(self.f)
        go = np.empty_like(self.g)
        lo = np.empty_like(self.lam)
        iters = np.empty(self.n, dtype=np.int32) if diagnostics else None
        eps = np.empty(self.n) if diagnostics else None
        tot = Stats()
        for _ in range(nsteps):
            st = Stats()
            self.L.orc_step(ctypes.byref(self.p), _ptr(self.f), _ptr(self.g), _ptr(self.lam), _ptr(fo), _ptr(go),
                           _ptr(lo), _ptr(iters), _ptr(eps), ctypes.byref(st))
            self.f, fo = fo, self.f
            self.g, go = go, self.g
            self.lam, lo = lo, self.lam
            tot.iterations += st.iterations
            tot.max_iterations = max(tot.max_iterations, st.max_iterations)
            tot.failed += st.failed
            tot.cold_restarts += st.cold_restarts
            tot.evaluations += st.evaluations
            for k in range(4):
                tot.alpha_hist[k] += st.alpha_hist[k]
        self.stats = tot
        if diagnostics:
            return iters, eps
        return None

    def stream_only(self, h):
        h = np.ascontiguousarray(h, dtype=np.float64).reshape(-1)
        out = np.empty_like(h)
        self.L.orc_stream_only(ctypes.byref(self.p), _ptr(h), _ptr(out))
        return out

    def moments(self):
        out = np.empty(5 * self.n)
        tot = np.empty(5)
        self.L.orc_moments(ctypes.byref(self.p), _ptr(self.f), _ptr(self.g), _ptr(out), _ptr(tot))
        return out.reshape(5, self.n), tot

    def cell_types(self):
        out = np.empty(self.n, dtype=np.uint8)
        self.L.orc_cell_types(ctypes.byref(self.p), _ptr(out))
        return out
