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


def branch_switch_bound(h_in, h_out_orc, eps_orc, eps_gpu, tau):
    """Per-population bound (39 x N) on |h'_gpu - h'_orc| that a different
    branch of Eq. (eq:alpha) alone causes: the relaxation h' = h + omega
    (h^eq - h) then differs by |omega_gpu - omega_orc| |h^eq - h|, with
    h^eq - h recovered from the oracle's own update.  Zero where the
    branches agree."""
    thr = np.array([1e-2, 1e-1, 1.0])
    om = np.array([1.0 / tau, 1.0 / (1.05 * tau), 1.0 / (1.35 * tau), 1.0])
    bo = np.digitize(np.nan_to_num(eps_orc, nan=-1.0), thr)
    bg = np.digitize(np.nan_to_num(eps_gpu, nan=-1.0), thr)
    wo, wg = om[bo], om[bg]
    d = (h_out_orc - h_in) / wo[None, :]
    return np.abs(wg - wo)[None, :] * np.abs(d)


def shift_weights(orc, storage, shift, u_ref, T0, gamma):
    """The weights the library shifts stored populations by (the rest or the
    stream equilibrium, on the 2^-21 grid) and the power-of-two shell scales
    of FP16 storage (ones otherwise): (w_f, w_g, s_f, s_g), 39 each."""
    rest_f, _, _, _ = orc.equilibrium(1.0, [0.0, 0.0, 0.0], T0, gamma=gamma, tol=1e-14, maxit=200)
    w_f = rest_f
    if shift:
        w_f, _, _, _ = orc.equilibrium(1.0, u_ref, T0, gamma=gamma, tol=1e-14, maxit=200)
    delta = 2.0 / (gamma - 1.0) - 3.0
    w_f = np.round(w_f * 2.0 ** 21) / 2.0 ** 21
    w_g = np.round(delta * T0 * w_f * 2.0 ** 21) / 2.0 ** 21
    if storage != "fp16s":
        return w_f, w_g, np.ones(39), np.ones(39)
    c = orc.velocities()
    q = (c ** 2).sum(1)
    s_f = np.array([2.0 ** np.round(np.log2(rest_f[np.flatnonzero(q == qq)[0]])) for qq in q])
    s_g = s_f * 2.0 ** np.round(np.log2(delta * T0))
    return w_f, w_g, s_f, s_g


def fp16_moment_bound(orc, f_in, f_out, g_in, g_out, w_f, w_g, s_f, s_g, mo, gamma, roundings=2, rel=1e-5):
    """Per-cell bounds (rho, |u|, T) on the moment error of an FP16-shifted
    step against the oracle: each stored population is off by at most
    2^-11 |h_i - w_i| + 2^-25 s_i per rounding (roundings: the gathered value
    and the written one, plus a re-encoding of bounced values), while the
    collision itself conserves mass, momentum and energy to FP32 rounding
    (rel of the cell's moments).  Propagated to first order into
    u = j / rho and T = (E - rho |u|^2) / (2 C_v rho).  Arrays 39 x N for
    the populations and 5 x N for mo (the oracle's moments)."""
    xi = orc.velocities().astype(np.float64)
    q = (xi ** 2).sum(1)

    def dev(h, w, s):
        return 2.0 ** -11 * np.abs(h - w[:, None]) + 2.0 ** -25 * s[:, None]

    df = (roundings - 1) * dev(f_in, w_f, s_f) + dev(f_out, w_f, s_f)
    dg = (roundings - 1) * dev(g_in, w_g, s_g) + dev(g_out, w_g, s_g)
    rho, u, T = mo[0], mo[1:4], mo[4]
    speed = np.sqrt((u ** 2).sum(0))
    two_cv = 2.0 / (gamma - 1.0)
    b_rho = df.sum(0) + rel * rho
    b_j = (df * np.sqrt(q)[:, None]).sum(0) + rel * rho
    b_e = (df * q[:, None]).sum(0) + dg.sum(0) + rel * rho * (speed ** 2 + two_cv * T)
    b_u = (b_j + speed * b_rho) / rho
    b_T = (b_e + 2.0 * speed * b_j + (speed ** 2 + two_cv * T) * b_rho) / (two_cv * rho)
    return b_rho, b_u, b_T


def moment_errors_over_bound(m, mo, bounds, cells):
    """Largest per-cell moment error divided by its bound (rho, |u|, T)."""
    b_rho, b_u, b_T = bounds
    e_rho = np.abs(m[0, cells] - mo[0, cells])
    e_u = np.sqrt(((m[1:4, cells] - mo[1:4, cells]) ** 2).sum(0))
    e_T = np.abs(m[4, cells] - mo[4, cells])
    return float(max((e_rho / b_rho[cells]).max(), (e_u / b_u[cells]).max(), (e_T / b_T[cells]).max()))
