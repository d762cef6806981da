"""The step at the largest grids the library takes, in every storage mode.

The kernels address a solve's populations with 32-bit byte offsets from
per-plane bases where they can: an FP32 gather reaches across a velocity
pair (2 planes of 4n bytes), an FP64 or FP16 gather across one velocity's
plane of paired records (16n and 4n bytes), so lbm_create takes fewer than
2^28 cells in FP64, 2^29 in FP32 and 2^30 in FP16.  The FP32 and FP16 row
stores span 4 planes of 4n bytes; above 2^28 cells they switch from a 32-bit
lane offset to a 64-bit lane address.  Device
memory bounds every mode before its offset bound (FP64 at 1.4 kB per cell,
FP32 at 0.68 kB, FP16 at 0.42 kB).

Here each mode runs at the largest grid that fits 80% of the free device
memory: 136 x 1024 x nz cells (rows of two full 64-cell segments, which take
the row stores, and a ragged 8-cell one), with nz a multiple of 4.  FP32 and
FP16 must land above 2^28 cells, in the 64-bit store path.  The initial fields
repeat with period (136, 4, 4), and every axis is periodic, so the exact
result is periodic too.  The check:

* every (136, 4, 4) tile of the result equals the first, bit for bit: a wrong
  offset anywhere in the grid would read other planes or other rows;
* the first tile matches the oracle on the (136, 4, 4) box, at the
  reduced-precision bars of two steps (FP64: 1e-12)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from _helpers import moment_error  # noqa: E402

from paper_1910_13515_amd import inputs  # noqa: E402

TILE = (136, 4, 4)
NY = 1024
# the gathers' offset bound per mode (cells)
MAX_CELLS = {"fp64": 1 << 28, "fp32s": 1 << 29, "fp16s": 1 << 30}
WIDE = 1 << 28  # from here on the FP32 and FP16 row stores use 64-bit lane addresses
STEPS = 2
# moment bars after two steps: twice the single-step bars of the
# reduced-precision modes; FP64 at the parity bar
BARS = {"fp64": 1e-12, "fp32s": 2 * 3e-5, "fp16s": 2 * 1e-3}


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


def _largest_nz(lbm, storage, budget):
    nz = (MAX_CELLS[storage] - 1) // (TILE[0] * NY) // 4 * 4
    while nz >= 4:
        try:
            need = lbm.lbm_required_bytes(lbm.make_params((TILE[0], NY, nz), storage=storage, tau=0.6))
        except lbm.LbmError:
            need = None
        if need is not None and need <= budget:
            return nz, need
        nz -= 4
    return 0, 0


@pytest.mark.parametrize("storage", ["fp32s", "fp16s", "fp64"])
def test_largest_grid_step(orc, lbm, storage):
    import torch
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    nz, need = _largest_nz(lbm, storage, int(0.8 * free))
    if nz < 4:
        pytest.skip(f"{free / 2**30:.1f} GiB free on the device")
    nx, ny = TILE[0], NY
    n = nx * ny * nz
    _log(f"largest grid {storage}: {nx} x {ny} x {nz} = {n} cells ({n / WIDE:.4f} of 2^28), "
         f"{need / 2**30:.1f} GiB")
    if storage != "fp64":
        assert n > WIDE  # the 64-bit row-store path is what is tested
    rho_t, u_t, T_t = inputs.random_fields(TILE, seed=11, rho=(0.9, 1.1), umax=0.15, T=(0.45, 0.55))
    reps = (nz // TILE[2], ny // TILE[1], 1)
    rho = np.tile(rho_t.reshape(TILE[::-1]), reps).reshape(-1)
    T = np.tile(T_t.reshape(TILE[::-1]), reps).reshape(-1)
    u = np.tile(u_t.reshape((3,) + TILE[::-1]), (1,) + reps).reshape(3, -1)
    kw = dict(gamma=1.4, tau=0.6, kn_relax=True)
    if storage == "fp64":
        kw.update(newton_tol=1e-13, newton_maxit=30)  # the oracle's threshold, as in every FP64 parity test
    s = lbm.Solver((nx, ny, nz), fields=(rho, u, T), storage=storage, **kw)
    del rho, u, T
    s.step(STEPS - 1)
    st = s.step(1, stats=True)
    m, tot = s.moments()
    s.close()
    del s
    torch.cuda.empty_cache()
    _log(f"  stepped; Newton failures {st.failed}")
    assert st.failed == 0
    assert np.all(np.isfinite(tot))
    view = m.reshape(5, nz // TILE[2], TILE[2], ny // TILE[1], TILE[1], nx)
    first = view[:, :1, :, :1, :, :]
    for k in range(5):
        assert np.array_equal(view[k], np.broadcast_to(first[k], view[k].shape)), k
    tile = np.ascontiguousarray(first).reshape(5, -1)
    del m, view
    o = orc.Oracle(*TILE, gamma=1.4, tau=0.6, kn_relax=True, newton_tol=1e-13, newton_maxit=30)
    assert o.init(rho_t, u_t, T_t) == 0
    o.step(STEPS)
    mo, _ = o.moments()
    em = moment_error(tile, mo)
    _log(f"  tiles identical; first tile against the oracle: rho {em[0]:.2e} u {em[1]:.2e} T {em[2]:.2e}")
    assert max(em) < BARS[storage]
