"""The seeded input generators (host only): the workloads' geometry and
fields, and the serving trace's envelope."""
import math

import numpy as np

from paper_1910_13515_amd import inputs


def test_taylor_green_fields_are_divergence_free_with_the_stated_pressure():
    n, U, T0 = 32, 0.4183, 0.5
    rho, u, T = inputs.taylor_green_fields(n, U, T0)
    ux, uy, uz = (c.reshape(n, n, n) for c in u)  # [z][y][x]
    k = 2 * math.pi / n
    # spectral derivatives are exact for the single-mode field
    kx = np.fft.fftfreq(n, d=1.0 / n) * k
    dux = np.real(np.fft.ifft(1j * kx[None, None, :] * np.fft.fft(ux, axis=2), axis=2))
    duy = np.real(np.fft.ifft(1j * kx[None, :, None] * np.fft.fft(uy, axis=1), axis=1))
    assert np.max(np.abs(dux + duy)) < 1e-13
    assert np.all(uz == 0.0)
    assert abs(np.max(np.abs(ux)) - U) < 1e-12
    np.testing.assert_allclose(T, T0)
    x = (np.arange(n ** 3) % n) * k
    y = ((np.arange(n ** 3) // n) % n) * k
    z = (np.arange(n ** 3) // (n * n)) * k
    p = T0 + U * U / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    np.testing.assert_allclose(rho * T, p, rtol=1e-14)


def test_naca_mask_has_the_profile_thickness():
    nx, ny, chord = 1024, 512, 256.0
    m = inputs.naca_symmetric_mask(nx, ny, 1, chord, 0.12, leading_edge=(nx / 2.0, ny / 2.0)).reshape(ny, nx)
    cols = np.flatnonzero(m.any(axis=0))
    assert cols[0] == nx // 2 and abs((cols[-1] - cols[0]) - chord) <= 1
    # thickest at 30% of the chord (inside the plateau of the voxelised
    # maximum): 12% of the chord, within a cell
    thick = m.sum(axis=0)
    top = np.flatnonzero(thick == thick.max())
    assert top[0] <= nx / 2 + 0.30 * chord <= top[-1]
    assert abs(thick.max() - 0.12 * chord) <= 1.5
    # symmetric about the chord line y = ny/2 (nodes at integer y)
    c = ny // 2
    np.testing.assert_array_equal(m[c + 1:ny], m[c - 1:0:-1])


def test_sphere_mask_volume():
    n, r = 96, 20.0
    m = inputs.sphere_mask(n, n, n, (48.0, 48.0, 48.0), r)
    assert abs(m.sum() / (4.0 / 3.0 * math.pi * r ** 3) - 1.0) < 0.01


def test_serving_trace_is_seeded_and_inside_its_envelope():
    # sizes and draws at the mix's own ranges, without fields
    for r in inputs.serving_trace(7, 200, 3.0, with_fields=False):
        n = r.shape[0]
        assert (200 <= n <= 4000) if r.kind == "tube" else (64 <= n <= 192)
    # fields on small boxes, so that the test stays quick
    a = inputs.serving_trace(7, 60, 3.0, box_cells=(16, 24))
    b = inputs.serving_trace(7, 60, 3.0, box_cells=(16, 24))
    assert [(r.kind, r.shape, r.steps, r.arrival) for r in a] == [(r.kind, r.shape, r.steps, r.arrival) for r in b]
    arrivals = np.array([r.arrival for r in a])
    assert np.all(np.diff(arrivals) > 0)
    assert 0.3 < np.mean(np.diff(arrivals)) < 0.4 + 0.3  # mean gap 1/3 s, loosely for 60 draws
    for r in a:
        assert 200 <= r.steps <= 2000 and 1e3 <= r.reynolds <= 1e4
        if r.kind == "tube":
            nx = r.shape[0]
            assert 200 <= nx <= 4000 and r.shape[1:] == (1, 1)
            rho_l, rho_r = r.rho[0], r.rho[-1]
            p_l, p_r = rho_l * r.T[0], rho_r * r.T[-1]
            rr, pr = rho_l / rho_r, p_l / p_r
            assert 2.0 - 1e-12 <= rr <= 10.0 + 1e-12
            assert rr - 1e-9 <= pr <= min(10.0, 3.2 * rr) + 1e-9   # the dense side is never the colder one
            assert abs(max(r.T[0], r.T[-1]) - 0.8) < 1e-12        # hot side at 0.8
            assert max(r.T) / min(r.T) <= 3.2 + 1e-9
            assert np.all(r.u == 0.0)
        else:
            nb = r.shape[0]
            assert 16 <= nb <= 24 and r.shape == (nb, nb, nb)
            assert 0.3 <= r.mach <= 1.5
            umax = r.mach * math.sqrt(1.4 * 0.5)
            assert abs(np.sqrt((r.u ** 2).sum(0)).max() - umax) < 1e-9 * umax or \
                abs(np.abs(r.u).max() - umax) < 1e-9 * umax
            np.testing.assert_allclose(r.T, 0.5)
