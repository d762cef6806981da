"""Stability of plain BGK against BGK with the Knudsen-number-based relaxation
on the supersonic NACA0012 flow (Sec. 4), held as stable or unstable outcomes.

Sec. 4 states three things about this flow:
  * plain BGK with the equilibrium of Eq. (eq:discrete-equilibrium) is stable
    up to Mach 1.2 and Reynolds 7500;
  * the relaxation factor alpha(eps) of Eq. (eq:alpha) extends that to Mach
    1.5 at Reynolds 1e4;
  * with alpha(eps), an under-resolved run at Reynolds 1e9 stays stable.

A run is "stable" when it stays finite and no cell update lacks an
equilibrium in its second half (the impulsive start may leave a few cells
without one).  "Unstable" means the flow keeps leaving the range where the
13-moment equilibrium exists: more than 0.1% of a chunk's updates fail after
the first quarter of the run, which is where the sweep stops it.  The full
sweep over (Ma, Re) is ``python -m paper_1910_13515_amd.stability_map``; these
are the cells that fit a test's time.  At half size (chord 128) the flow is
less resolved than at full size (chord 256), and plain BGK fails there even
at Ma 1.2 / Re 7500, so that statement is held at full size.
"""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1910_13515_amd import lbm as L
    return L


def _run(mach, reynolds, kn_relax, steps, scale):
    from paper_1910_13515_amd import stability_map
    _log(f"airfoil scale {scale}: Ma {mach} Re {reynolds:g} alpha(eps) {'on' if kn_relax else 'off'}, {steps} steps")
    r = stability_map.run_case(mach, reynolds, kn_relax, steps, scale, "fp64")
    _log(str(r))
    return r


def test_knudsen_relaxation_carries_mach_1_5_at_re_1e4(lbm):
    """BGK(eps) at Ma 1.5 / Re 1e4 (half size, 4000 steps): stable."""
    r = _run(1.5, 1e4, True, 4000, 0.5)
    assert r["finite"] and r["steps_run"] == 4000
    assert r["failed_second_half"] == 0
    assert r["stable"]


def test_plain_bgk_fails_at_mach_1_5_re_1e4(lbm):
    """Plain BGK at Ma 1.5 / Re 1e4 (half size): past the first quarter more
    than 0.1% of the updates find no equilibrium, chunk after chunk, and the
    sweep's rule stops the run."""
    steps = 2000
    r = _run(1.5, 1e4, False, steps, 0.5)
    n = 1024 * 512
    assert not r["stable"]
    assert r["steps_run"] < steps
    assert r["failed_first_half"] + r["failed_second_half"] > 1e-3 * n * (r["steps_run"] - steps // 4)


def test_plain_bgk_holds_at_mach_1_2_re_7500(lbm):
    """Plain BGK at Ma 1.2 / Re 7500, full size (chord 256, 6000 steps):
    stable, the paper's plain-BGK limit."""
    r = _run(1.2, 7500.0, False, 6000, 1.0)
    assert r["finite"] and r["steps_run"] == 6000
    assert r["failed_second_half"] == 0
    assert r["failed_first_half"] < 1e-6 * 2048 * 1024 * 3000
    assert r["stable"]


def test_under_resolved_re_1e9_stays_stable(lbm):
    """BGK(eps) at Ma 1.5 and Re 1e9 (tau - 1/2 = 6.5e-7) on the full-size
    grid, 4000 steps: stable."""
    r = _run(1.5, 1e9, True, 4000, 1.0)
    assert r["tau"] - 0.5 < 1e-6
    assert r["finite"] and r["steps_run"] == 4000
    assert r["failed_first_half"] == 0 and r["failed_second_half"] == 0
