"""GPU parity of the secant root finder (root_finder 1, FP64 storage) against
the oracle's secant solver (needs an MI355X).

The variant never evaluates the Jacobian of G: limited-memory BFGS on the
convex dual, started from the inverse of a model Jacobian (the rest Jacobian
at T_ref, scaled to the cell's temperature and shifted to its velocity).  The
oracle implements the same algorithm independently (model Jacobian built from
its definition and inverted by Cholesky; the kernel applies it factor by
factor), and is pinned on the CPU (tests/test_oracle_secant.py).  Bar: in
cells that take the same number of updates on both sides, 1e-12 relative on
every population (the same iterates; what remains is summation order); in
the others, the stop-rule bound of two iterates of the same root (see
_check_step and ITER_SHARE).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from _helpers import max_rel, moment_error, oracle_state  # noqa: E402

from paper_1910_13515_amd import inputs  # noqa: E402

TOL = 1e-12
# the share of cells whose update count may differ between the two
# implementations, and by how much.  Near the root of an ill-conditioned
# cell (a supersonic stream, condition ~5e3) the quasi-Newton direction often
# does not lower ||G||_2, and the step is taken on the dual objective's
# Armijo test, whose decrease there is of the order of the rounding of Phi
# (~1e-16): each side's rounding then decides whether a trial is taken, and
# the paths part by a few updates (the CPU prototype fails a quarter of such
# cells if those decisions are withheld).  Both sides still stop within the
# bound of the same root, which is what the populations are held to.
ITER_SHARE = 0.15
ITER_DIFF = 4


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_1910_13515_amd import lbm as L
    L.load()
    return L


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(orc, lbm, shape, T_ref=0.5, tau=0.55, kn=True, faces=(0,) * 6, solid=None, tol=1e-13, maxit=100,
          solver="secant"):
    o = orc.Oracle(*shape, gamma=1.4, tau=tau, kn_relax=kn, faces=faces, solid=solid, newton_tol=tol,
                   newton_maxit=maxit, root_finder=1 if solver == "secant" else 0, model_T=T_ref)
    s = lbm.Solver(shape, solid=solid, storage="fp64", gamma=1.4, tau=tau, kn_relax=kn, faces=faces, newton_tol=tol,
                   newton_maxit=maxit, T_ref=T_ref, root_finder=solver)
    return o, s


def _check_step(orc, o, s, tol=1e-13, iter_share=None, iter_diff=None):
    """One step on both sides.  Every fluid cell's populations must lie
    within what two iterates of the same root, each within the stopping
    bound, can differ by after the collision: omega times the difference of
    their equilibria, at most 2 omega eta_i f^eq_i with eta_i the stopping
    rule's relative error bound of f^eq_i (omega <= 2), plus TOL of the
    array maximum for summation order.  Cells that take the same number of
    updates on both sides usually follow the same iterates; they are held
    to 10 TOL (an acceptance decided by rounding mid-path can re-join).
    Then the update counts: at most iter_share of the cells may differ,
    none by more than iter_diff.  Returns (stats, GPU counts, oracle
    counts)."""
    from test_gpu_sensor import _basis, _newton_stop_error
    iter_share = ITER_SHARE if iter_share is None else iter_share
    iter_diff = ITER_DIFF if iter_diff is None else iter_diff
    _, it_g = s.diagnostics()
    it_o, _ = o.step(1, diagnostics=True)
    st = s.step(1, stats=True)
    n = s.n
    assert np.all((it_g == -1) == (it_o == -1))
    fluid = it_o >= 0
    same = it_g == it_o
    fg, gg, _ = s.get_state()
    fo, go = o.f.reshape(39, n), o.g.reshape(39, n)
    fg, gg = fg.reshape(39, n), gg.reshape(39, n)
    scale_f, scale_g = np.max(np.abs(fo)), np.max(np.abs(go))
    assert np.max(np.abs(fg - fo)[:, same]) <= 10 * TOL * scale_f
    assert np.max(np.abs(gg - go)[:, same]) <= 10 * TOL * scale_g
    solved = fluid & np.isfinite(o.lam.reshape(13, n)[0])
    lam = o.lam.reshape(13, n)[:, solved]
    eta = _newton_stop_error(orc, lam, tol, o.gamma)
    mo, _ = o.moments()
    feq = np.exp(_basis(orc) @ lam) * mo[0][solved][None, :]
    delta = 2.0 / (o.gamma - 1.0) - 3.0  # g^eq = delta T f^eq
    df = 2.0 * 2.0 * eta * feq
    assert np.all(np.abs(fg - fo)[:, solved] <= df + TOL * scale_f)
    assert np.all(np.abs(gg - go)[:, solved] <= df * (delta * mo[4][solved])[None, :] + TOL * scale_g)
    diff = np.abs(it_g - it_o)[fluid]
    assert np.mean(~same[fluid]) <= iter_share and np.all(diff <= iter_diff), (np.mean(~same[fluid]), diff.max())
    return st, it_g, it_o


def _stream_state(orc, shape, mach, T0, seed, amp=0.03):
    """A perturbed uniform stream along x (oracle-built)."""
    n = int(np.prod(shape))
    U = mach * np.sqrt(1.4 * T0)
    rho, u, T = inputs.random_fields(shape, seed=seed, rho=(0.95, 1.05), umax=0.05 * max(U, 0.2),
                                     T=(0.97 * T0, 1.03 * T0))
    u = u.reshape(3, n)
    u[0] += U
    o = orc.Oracle(*shape, gamma=1.4)
    assert o.init(rho, u.reshape(-1), T) == 0
    pert = inputs.random_perturbation(shape, seed=seed + 1, amplitudes=(amp,))
    return o.f * np.exp(pert[0].reshape(-1)), o.g * np.exp(pert[1].reshape(-1)), o.lam.copy()


@pytest.mark.parametrize("shape,amps", [((70, 5, 4), (1e-3, 3e-2, 0.3)), ((130, 3, 2), (1e-2,))])
def test_single_step_from_oracle_state(orc, lbm, shape, amps):
    _log(f"secant single step {shape}")
    f, g, lam = oracle_state(orc, shape, 1.4, seed=71, amplitudes=amps)
    o, s = _pair(orc, lbm, shape)
    o.set_state(f, g, lam)
    s.set_state(f, g, lam)
    st, it_g, it_o = _check_step(orc, o, s)
    m, _ = s.moments()
    mo, _ = o.moments()
    assert max(moment_error(m, mo)) < TOL
    assert st.failed == 0 and o.stats.failed == 0
    assert list(st.alpha_hist) == list(o.stats.alpha_hist)
    _log(f"  secant updates GPU {st.iterations} oracle {o.stats.iterations} over {np.prod(shape)} cells, "
         f"{int(np.sum(it_g != it_o))} cells differ")
    s.close()


@pytest.mark.parametrize("mach", [0.3, 1.2])
def test_obstacle_and_open_faces_in_a_stream(orc, lbm, mach):
    """Three steps of a perturbed stream past a sphere with equilibrium and
    Neumann faces, T_ref 2/3 (the model Jacobian is built there)."""
    shape = (40, 20, 6)
    _log(f"secant obstacle + faces, Ma {mach}")
    T0 = 2.0 / 3.0
    solid = inputs.sphere_mask(*shape, center=(18.5, 9.5, 2.5), radius=4.2)
    faces = (orc.FACE_EQUILIBRIUM, orc.FACE_NEUMANN, orc.FACE_EQUILIBRIUM, orc.FACE_EQUILIBRIUM, 0, 0)
    f, g, lam = _stream_state(orc, shape, mach, T0, seed=81)
    o, s = _pair(orc, lbm, shape, T_ref=T0, faces=faces, solid=solid)
    o.set_state(f, g, lam)
    s.set_state(f, g, lam)
    for k in range(3):
        st, it_g, it_o = _check_step(orc, o, s)
        assert st.failed == o.stats.failed == 0
        _log(f"  step {k}: updates GPU {st.iterations} oracle {o.stats.iterations}, "
             f"{int(np.sum(it_g != it_o))} cells differ")
    m, t = s.moments()
    mo, to = o.moments()
    assert max(moment_error(m, mo)) < TOL
    # totals (mass, momentum, energy) relative to the largest one: a
    # near-zero momentum total carries the other cells' stop differences
    np.testing.assert_allclose(t, to, rtol=0, atol=1e-12 * np.max(np.abs(to)))
    s.close()


def test_secant_step_equals_newton_step(orc, lbm):
    """The variant changes how the equilibrium is found, not what it is: on
    the GPU the secant and Newton steps agree within the stopping bound."""
    shape = (70, 5, 4)
    f, g, lam = oracle_state(orc, shape, 1.4, seed=91, amplitudes=(1e-3, 3e-2, 0.3))
    out = {}
    for solver in ("newton", "secant"):
        _, s = _pair(orc, lbm, shape, solver=solver)
        s.set_state(f, g, lam)
        st = s.step(2, stats=True)
        out[solver] = (s.get_state(), st.iterations)
        s.close()
    (fa, ga, _), ita = out["newton"]
    (fb, gb, _), itb = out["secant"]
    assert max_rel(fb, fa) < 1e-11
    assert max_rel(gb, ga) < 1e-11
    _log(f"  updates over 2 steps: Newton {ita}, secant {itb}")
    assert itb > ita


def test_diagnostics_match_oracle(orc, lbm):
    """Per-cell sensor and secant update counts of the next step."""
    shape = (70, 5, 4)
    f, g, lam = oracle_state(orc, shape, 1.4, seed=101, amplitudes=(1e-3, 3e-2, 0.3))
    o, s = _pair(orc, lbm, shape)
    o.set_state(f, g, lam)
    s.set_state(f, g, lam)
    eps_g, it_g = s.diagnostics()
    it_o, eps_o = o.step(1, diagnostics=True)
    ok = ~np.isnan(eps_o)
    np.testing.assert_array_equal(np.isnan(eps_g), np.isnan(eps_o))
    same = (it_g == it_o) & ok
    assert np.max(np.abs(eps_g[same] - eps_o[same]) / np.abs(eps_o[same])) < 1e-10
    assert np.mean(it_g[ok] != it_o[ok]) <= ITER_SHARE
    assert np.all(np.abs(it_g[ok] - it_o[ok]) <= ITER_DIFF)
    thr = [1e-2, 1e-1, 1.0]
    np.testing.assert_array_equal(np.digitize(eps_g[ok], thr), np.digitize(eps_o[ok], thr))
    s.close()


def test_cells_without_equilibrium_are_marked(orc, lbm):
    """A slab whose moments have no equilibrium: the secant solver fails
    there as the oracle's does; such cells are not collided, lambda_0 is
    NaN, the rest of the grid matches."""
    shape = (16, 4, 4)
    n = int(np.prod(shape))
    rho, u, T = inputs.uniform_fields(n, 1.0, [0.1, 0.0, 0.0], 0.5)
    o, s = _pair(orc, lbm, shape, maxit=60)
    assert o.init(rho, u, T) == 0
    f, g, lam = o.f.copy(), o.g.copy(), o.lam.copy()
    c = orc.velocities()
    q = (c ** 2).sum(1)
    G = g.reshape(39, n).copy()
    x = np.arange(n) % shape[0]
    cold = (x >= 2) & (x <= 9)  # a slab across x, as in the Newton test
    e_now = (f.reshape(39, n) * q[:, None]).sum(0) + G.sum(0)
    G[:, cold] += ((1.0 * 0.01 + 5.0 * 0.1 - e_now[cold]) / 39.0)[None, :]
    o.set_state(f, G.reshape(-1), lam)
    s.set_state(f, G.reshape(-1), lam)
    # step 1: the slab's cells away from its edges (which mix with the warm
    # neighbours in the gather) have no equilibrium; both sides fail on the
    # same cells, leave them uncollided and mark them
    st, it_g, it_o = _check_step(orc, o, s, iter_share=1.0, iter_diff=100)
    assert st.failed == o.stats.failed > 0
    assert st.cold_restarts == o.stats.cold_restarts
    _, _, lg = s.get_state()
    np.testing.assert_array_equal(np.isnan(lg.reshape(13, n)[0]), np.isnan(o.lam.reshape(13, n)[0]))
    # step 2: after one uncollided step the slab's edge cells have mixed with
    # their neighbours and sit at the edge of the equilibrium range, where a
    # secant path may or may not reach the root within the cap (a cell that
    # converged in step 1 and now fails its warm start is restarted cold); each
    # side's failures carry its mark
    st, it_g, it_o = _check_step(orc, o, s, iter_share=1.0, iter_diff=100)
    _log(f"  second step: failed cells GPU {st.failed}, oracle {o.stats.failed}")
    assert st.failed > 0 and o.stats.failed > 0
    _, _, lg = s.get_state()
    lam0_g = lg.reshape(13, n)[0]
    assert np.sum(np.isnan(lam0_g)) == st.failed
    assert np.sum(np.isnan(o.lam.reshape(13, n)[0])) == o.stats.failed
    s.close()


def test_tgv32_trajectory(orc, lbm):
    """20 steps of the 32^3 Taylor-Green vortex with the secant solver."""
    n = 32
    _log("secant TGV 32^3, 20 steps")
    U = 0.5 * np.sqrt(1.4 * 0.5)
    fields = inputs.taylor_green_fields(n, U, 0.5)
    s = lbm.Solver((n, n, n), fields=fields, storage="fp64", gamma=1.4, tau=0.52, newton_tol=1e-13,
                   newton_maxit=100, root_finder="secant")
    o = orc.Oracle(n, n, n, gamma=1.4, tau=0.52, newton_tol=1e-13, newton_maxit=100, root_finder=1, model_T=0.5)
    assert o.init(*fields) == 0
    for k in range(4):
        o.step(5)
        st = s.step(5, stats=True)
        m, _ = s.moments()
        mo, _ = o.moments()
        err = max(moment_error(m, mo))
        _log(f"  step {5 * (k + 1)}: moments {err:.2e}, updates GPU {st.iterations} oracle {o.stats.iterations}")
        assert err < TOL
    s.close()
