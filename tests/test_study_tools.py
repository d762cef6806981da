"""Host-side statistics of the study tools (no GPU): the airfoil's sensor and
iteration summary, and the error norms of the precision studies."""
import numpy as np

from paper_1910_13515_amd import knudsen_map, precision_study


def _fields(shape, solid):
    """A synthetic sensor/iteration field with a known composition: frozen
    face columns (x < 3 or x >= nx - 3, iterations -1), one failed cell, and
    eps/iterations set by the x coordinate."""
    nx, ny, _ = shape
    n = nx * ny
    x = np.arange(n) % nx
    eps = np.where(x < nx // 2, 1e-6, 0.05)
    eps = np.where(x >= nx - nx // 8, 0.5, eps)
    iters = np.where(x < nx // 2, 0.0, 2.0)
    frozen = (x < 3) | (x >= nx - 3)
    iters[frozen] = -1.0
    eps[frozen] = np.nan
    sol = solid.reshape(-1) != 0
    iters[sol] = -1.0
    eps[sol] = np.nan
    failed = np.flatnonzero(~frozen & ~sol)[7]
    eps[failed] = np.nan
    iters[failed] = 20.0
    return eps, iters, frozen, sol, failed, x


def test_knudsen_summary_counts():
    shape, solid, _ = precision_study.airfoil_case(0.125)
    eps, iters, frozen, sol, failed, x = _fields(shape, solid)
    res = knudsen_map.summarize(shape, solid, eps, iters)
    upd = ~frozen & ~sol
    assert res["updated_cells"] == int(upd.sum())
    nu = res["newton_updates"]
    assert nu["cells_without_equilibrium"] == 1
    ok = upd.copy()
    ok[failed] = False
    zero = ok & (x < shape[0] // 2)
    assert nu["histogram_0_to_4_and_more"][0] == int(zero.sum())
    assert nu["histogram_0_to_4_and_more"][2] == int((ok & ~zero).sum())
    assert nu["max"] == 2
    assert abs(nu["share_zero"] - zero.sum() / ok.sum()) < 1e-12
    shares = res["alpha_branch_share"]
    assert abs(sum(shares) - 1.0) < 1e-12
    b2 = ok & (x >= shape[0] - shape[0] // 8)
    assert abs(shares[2] - b2.sum() / ok.sum()) < 1e-12
    assert shares[3] == 0.0
    xr = res["sensor"]["active_x_range"]
    assert xr[0] == shape[0] // 2 and xr[1] == shape[0] - 4


def test_relative_l2_errors():
    rng = np.random.default_rng(3)
    ref = rng.uniform(0.5, 1.5, (5, 100))
    f = ref.copy()
    f[0] *= 1.0 + 1e-3
    fluid = np.ones(100, dtype=bool)
    e = precision_study.errors(f, ref, fluid)
    assert abs(e["l2_rho"] - 1e-3) < 1e-12
    assert e["l2_u"] == 0.0 and e["l2_T"] == 0.0
    assert abs(e["max_rho"] - np.max(np.abs(ref[0]) * 1e-3)) < 1e-15


def test_precision_study_mode_strings():
    import pytest
    ps = precision_study
    assert ps.parse_mode("fp64") == ("fp64", 0, 0.0)
    assert ps.parse_mode("fp32s@stream") == ("fp32s", 1, 0.0)
    assert ps.parse_mode("fp64:1e-13") == ("fp64", 0, 1e-13)
    assert ps.parse_mode("fp16s@stream:2e-6") == ("fp16s", 1, 2e-6)
    for bad in ("fp8", "fp32s@rest", "fp64@stream"):
        with pytest.raises(ValueError):
            ps.parse_mode(bad)


def test_bow_shock_position_on_a_row():
    """The shock's mid-point on a synthetic density row: free stream 1 up to
    x = 40, a linear rise to 2.2 over x = 40..44 and a plateau; the half
    level 1.6 is crossed at x = 42, interpolated between cells."""
    shape = (128, 5, 1)
    rho = np.ones(shape[::-1])
    x = np.arange(shape[0])
    row = np.clip(1.0 + 0.3 * (x - 40), 1.0, 2.2)
    rho[0, 2, :] = row
    assert abs(precision_study.shock_front(rho, shape, 100, 2) - 42.0) < 1e-12
    # no rise, or a row whose maximum is within 1% of the free stream: none
    assert np.isnan(precision_study.shock_front(rho, shape, 100, 0))
    rho[0, 1, 50:] = 1.005
    assert np.isnan(precision_study.shock_front(rho, shape, 100, 1))


def test_shock_rows_stop_at_the_body():
    """The rows scanned for the bow shock end at the body: the airfoil's
    stagnation row at its leading edge (the domain centre), the sphere's rows
    where they meet the sphere."""
    x0, rows = precision_study.front_rows("airfoil", (2048, 1024, 1), 1.0)
    assert x0 == 1024 and rows[0] == ("stagnation", 512, 0, 1024)
    _, solid, _ = precision_study.airfoil_case(1.0)
    sm = solid.reshape(1, 1024, 2048)
    for _, y, z, xe in rows:
        assert not sm[z, y, :xe].any()
    shape = (128, 64, 64)
    x0, rows = precision_study.front_rows("sphere", shape, 0.25)
    _, ssolid, _ = precision_study.sphere_case(0.25)
    sm = ssolid.reshape(64, 64, 128)
    for _, y, z, xe in rows:
        assert not sm[z, y, :xe].any() and xe > 0
