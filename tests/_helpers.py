"""Shared helpers of the parity tests: oracle-built states and comparisons.
States always flow oracle -> library, never the other way."""
import numpy as np

from paper_1910_13515_amd import inputs


def oracle_state(orc, shape, gamma, seed, amplitudes=(1e-3, 3e-2, 0.3), spread=1.0, umax=0.2):
    """A random non-equilibrium state built by the oracle: equilibria of
    random fields times exp(random perturbation)."""
    nx, ny, nz = shape
    rho, u, T = inputs.random_fields(shape, seed=seed, rho=(1 - 0.2 * spread, 1 + 0.2 * spread), umax=umax * spread,
                                     T=(0.5 - 0.05 * spread, 0.5 + 0.1 * spread))
    o = orc.Oracle(nx, ny, nz, gamma=gamma)
    assert o.init(rho, u, T) == 0
    pert = inputs.random_perturbation(shape, seed=seed + 1, amplitudes=amplitudes)
    f = o.f * np.exp(pert[0].reshape(-1))
    g = o.g * np.exp(pert[1].reshape(-1))
    return f, g, o.lam.copy()


def max_rel(a, b, floor=None):
    """max |a - b| / max(|b|) (a scale-aware elementwise error)."""
    a = np.asarray(a)
    b = np.asarray(b)
    scale = np.max(np.abs(b)) if floor is None else floor
    return float(np.max(np.abs(a - b)) / scale)


def moment_error(m_gpu, m_orc):
    """Per-field relative error of (rho, u, T): rho and T relative to their
    values, u relative to the speed scale max(|u|, 1e-3)."""
    ok = np.isfinite(m_orc[0])
    rho = np.max(np.abs(m_gpu[0][ok] - m_orc[0][ok]) / np.abs(m_orc[0][ok]))
    T = np.max(np.abs(m_gpu[4][ok] - m_orc[4][ok]) / np.abs(m_orc[4][ok]))
    speed = max(np.max(np.sqrt((m_orc[1:4, ok] ** 2).sum(0))), 1e-3)
    u = np.max(np.abs(m_gpu[1:4, ok] - m_orc[1:4, ok])) / speed
    return float(rho), float(u), float(T)
