"""Seeded synthetic inputs for the D3Q39 solver and its checks.

This module holds only input generation: initial macroscopic fields, obstacle
masks, random numbers and request traces.  It contains none of the lattice
Boltzmann arithmetic (no equilibrium, streaming or collision), so both the
library's tests and the oracle's tests can draw the same inputs from it.

Every field is a float64 numpy array in x-fastest order (index x + nx*(y +
ny*z)); velocity fields are stacked SoA as [ux, uy, uz] (shape (3, N)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def grid_coords(nx: int, ny: int, nz: int):
    """Integer node coordinates (x, y, z), each of length nx*ny*nz."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def uniform_fields(n: int, rho: float, u, T: float):
    u = np.asarray(u, dtype=np.float64)
    return (np.full(n, float(rho)), np.repeat(u[:, None], n, axis=1).astype(np.float64), np.full(n, float(T)))


def sod_fields(nx: int, ny: int = 1, nz: int = 1, rho_l: float = 1.0, p_l: float = 1.0, rho_r: float = 0.125,
               p_r: float = 0.1, temp_scale: float = 0.5, split: int | None = None):
    """Shock-tube initial state: gas at rest, (rho_l, p_l) for x < split and
    (rho_r, p_r) beyond, the temperature p/rho multiplied by temp_scale to
    bring it into lattice units (velocities then scale by sqrt(temp_scale))."""
    split = nx // 2 if split is None else split
    x, _, _ = grid_coords(nx, ny, nz)
    left = x < split
    rho = np.where(left, rho_l, rho_r).astype(np.float64)
    p = np.where(left, p_l, p_r).astype(np.float64)
    T = temp_scale * p / rho
    u = np.zeros((3, nx * ny * nz))
    return rho, u, T


def taylor_green_fields(n: int, amplitude: float, T0: float, p0: float | None = None):
    """Compressible Taylor-Green vortex on a periodic n^3 grid with nodes at
    integer positions: u = U sin kx cos ky cos kz, v = -U cos kx sin ky cos kz,
    w = 0, p = p0 + rho0 U^2/16 (cos 2kx + cos 2ky)(cos 2kz + 2), uniform
    temperature T0 and rho = p / T0 (rho0 = 1, p0 = T0 by default)."""
    k = 2.0 * math.pi / n
    x, y, z = grid_coords(n, n, n)
    x, y, z = k * x, k * y, k * z
    U = amplitude
    rho0 = 1.0
    p0 = rho0 * T0 if p0 is None else p0
    ux = U * np.sin(x) * np.cos(y) * np.cos(z)
    uy = -U * np.cos(x) * np.sin(y) * np.cos(z)
    uz = np.zeros_like(ux)
    p = p0 + rho0 * U * U / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    T = np.full_like(ux, T0)
    rho = p / T0
    return rho, np.stack([ux, uy, uz]), T


def naca_symmetric_mask(nx: int, ny: int, nz: int, chord: float, thickness: float = 0.12,
                        leading_edge=None, closed_trailing_edge: bool = False):
    """Voxelised symmetric NACA 4-digit profile at zero incidence (extruded
    along z).  Half thickness y_t = 5 t c (0.2969 sqrt(s) - 0.1260 s - 0.3516 s^2
    + 0.2843 s^3 - c4 s^4) with s = (x - x0)/c, c4 = 0.1015 (open trailing edge)
    or 0.1036 (closed).  A node is solid when its centre lies inside."""
    x0, y0 = (nx / 2.0, ny / 2.0) if leading_edge is None else leading_edge
    c4 = 0.1036 if closed_trailing_edge else 0.1015
    x, y, _ = grid_coords(nx, ny, nz)
    s = (x.astype(np.float64) - x0) / chord
    inside = (s >= 0.0) & (s <= 1.0)
    sc = np.clip(s, 0.0, 1.0)
    yt = 5.0 * thickness * chord * (0.2969 * np.sqrt(sc) - 0.1260 * sc - 0.3516 * sc ** 2 + 0.2843 * sc ** 3
                                    - c4 * sc ** 4)
    solid = inside & (np.abs(y.astype(np.float64) - y0) <= yt)
    return solid.astype(np.uint8)


def sphere_mask(nx: int, ny: int, nz: int, center, radius: float):
    x, y, z = grid_coords(nx, ny, nz)
    d2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    return (d2 <= radius * radius).astype(np.uint8)


def random_fields(shape, seed: int, rho=(0.8, 1.2), umax: float = 0.3, T=(0.45, 0.6)):
    """Random smooth-free macroscopic fields: rho and T uniform in the given
    ranges, each velocity component uniform in [-umax, umax]."""
    nx, ny, nz = shape
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    r = rng.uniform(rho[0], rho[1], n)
    u = rng.uniform(-umax, umax, (3, n))
    t = rng.uniform(T[0], T[1], n)
    return r, u, t


def random_perturbation(shape, seed: int, q: int = 39, amplitudes=(1e-3, 3e-2, 0.3, 2.0)):
    """Random log-perturbation factors for non-equilibrium test states:
    returns a (2, q, N) array a_c * r with r uniform in [-1, 1], where a_c is
    drawn per cell from ``amplitudes`` (spanning every branch of the
    relaxation-factor table).  A caller forms h = h_eq * exp(factor)."""
    nx, ny, nz = shape
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    amp = rng.choice(np.asarray(amplitudes, dtype=np.float64), size=n)
    r = rng.uniform(-1.0, 1.0, (2, q, n))
    return r * amp[None, None, :]


def solenoidal_random_velocity(n: int, seed: int, umax: float, kmin: int = 1, kmax: int = 4):
    """Random-phase solenoidal velocity on a periodic n^3 grid with energy in
    shells kmin <= |k| <= kmax, spectrum E(k) ~ k^4 exp(-k^2/2), scaled so
    that max |u| = umax."""
    rng = np.random.default_rng(seed)
    kk = np.fft.fftfreq(n, d=1.0 / n)
    kx, ky, kz = np.meshgrid(kk, kk, kk, indexing="ij")
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    kmag = np.sqrt(k2)
    shell = (kmag >= kmin) & (kmag <= kmax)
    amp = np.where(shell, kmag ** 2 * np.exp(-k2 / 4.0), 0.0) / np.maximum(kmag, 1.0)
    comps = []
    for _ in range(3):
        phase = rng.uniform(0.0, 2.0 * np.pi, kx.shape)
        comps.append(amp * np.exp(1j * phase))
    a = np.stack(comps)
    # project out the compressive part: a - k (k.a)/|k|^2
    kvec = np.stack([kx, ky, kz])
    dot = (kvec * a).sum(0) / np.where(k2 > 0, k2, 1.0)
    a = a - kvec * dot[None]
    u = np.real(np.fft.ifftn(a, axes=(1, 2, 3)))
    # reorder from (x, y, z) indexing to x-fastest flat order
    u = np.transpose(u, (0, 3, 2, 1)).reshape(3, -1)
    m = np.sqrt((u ** 2).sum(0)).max()
    return u * (umax / m)


@dataclass
class Request:
    """One independent solve in a serving trace."""
    rid: int
    arrival: float          # seconds after the trace start
    kind: str               # "tube" or "box"
    shape: tuple
    steps: int
    gamma: float = 1.4
    mach: float = 0.0
    reynolds: float = 0.0
    tau: float = 0.0
    T_ref: float = 0.5      # reference temperature (relaxation time, shift weights)
    rho: np.ndarray = field(default=None, repr=False)
    u: np.ndarray = field(default=None, repr=False)
    T: np.ndarray = field(default=None, repr=False)


def serving_trace(seed: int, count: int, rate: float, T_ref: float = 0.5, gamma: float = 1.4,
                  tube_cells=(200, 4000), box_cells=(64, 192), steps=(200, 2000), ratio=(2.0, 10.0),
                  mach=(0.3, 1.5), reynolds=(1e3, 1e4), with_fields: bool = True, tube_T_hot: float = 0.8,
                  tube_T_ratio_max: float = 3.2):
    """Poisson arrivals (exponential gaps of mean 1/rate) of independent
    solves, half 1-D Riemann tubes (x periodic, left state denser and hotter
    by the drawn ratios) and half periodic 3-D boxes with a random-phase
    solenoidal velocity.  Box velocities are Ma sqrt(gamma T_ref) at their
    maximum, at uniform T_ref.

    Tubes stay inside the temperature window where the D3Q39 equilibrium
    exists along the whole run: the density ratio is drawn from ``ratio``, the
    pressure ratio from ``ratio`` limited to [density ratio, density ratio *
    tube_T_ratio_max] (the dense side is never the colder one, and the two
    temperatures differ by at most tube_T_ratio_max), and the hot side sits at
    tube_T_hot, which is also the tube's reference temperature.
    Relaxation times are left to the solver (``reynolds`` and the reference
    length n/2pi of a box or n/8 of a tube)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        if rng.uniform() < 0.5:
            nx = int(rng.integers(tube_cells[0], tube_cells[1] + 1))
            rr = rng.uniform(*ratio)
            pr = rng.uniform(max(rr, ratio[0]), min(ratio[1], rr * tube_T_ratio_max))
            re = float(np.exp(rng.uniform(np.log(reynolds[0]), np.log(reynolds[1]))))
            req = Request(rid, t, "tube", (nx, 1, 1), nsteps, gamma=gamma, mach=0.0, reynolds=re,
                          T_ref=tube_T_hot)
            if with_fields:
                # left state (rho, p) = (rr, pr), right (1, 1); T = s p / rho with the
                # left (hot) side at tube_T_hot
                s = tube_T_hot * rr / pr
                req.rho, req.u, req.T = sod_fields(nx, 1, 1, rho_l=rr, p_l=pr, rho_r=1.0, p_r=1.0, temp_scale=s)
        else:
            nb = int(rng.integers(box_cells[0], box_cells[1] + 1))
            ma = float(rng.uniform(*mach))
            re = float(np.exp(rng.uniform(np.log(reynolds[0]), np.log(reynolds[1]))))
            req = Request(rid, t, "box", (nb, nb, nb), nsteps, gamma=gamma, mach=ma, reynolds=re, T_ref=T_ref)
            if with_fields:
                umax = ma * math.sqrt(gamma * T_ref)
                u = solenoidal_random_velocity(nb, int(rng.integers(1 << 31)), umax)
                req.rho = np.ones(nb ** 3)
                req.u = u
                req.T = np.full(nb ** 3, T_ref)
        out.append(req)
    return out
