"""The seeded input generators: determinism, shapes, ranges and structure."""
import math

import numpy as np

import workloads as W


def test_small_binary_recipe():
    a, b = W.small_binary(0), W.small_binary(0)
    assert a.eps.dtype == np.float32 and a.eps.shape == (64, 64)
    assert np.array_equal(a.eps, b.eps) and np.array_equal(a.b, b.b)
    assert set(np.unique(a.eps)) <= {np.float32(2.085), np.float32(12.25)}
    assert np.all(a.eps[:16] == np.float32(2.085)) and np.all(a.eps[:, 48:] == np.float32(2.085))
    frac = np.mean(a.eps[16:48, 16:48] == np.float32(12.25))
    assert 0.4 < frac < 0.6
    J = (a.b / (-1j * a.omega)).reshape(64, 64)
    assert np.allclose(J[:, 12], 1.0) and np.count_nonzero(J) == 64
    assert abs(a.omega - 2 * math.pi / 1.55) < 1e-12


def test_grating_recipe():
    g = W.grating(1000)
    assert g.eps.shape == (240, 480) and g.npml == 20 and g.dx == 0.025
    assert g.eps.min() >= np.float32(2.085) and g.eps.max() <= np.float32(12.25)
    x0, y0, wx, wy = W.design_box(480, 240)
    assert (x0, y0, wx, wy) == (140, 80, 200, 80)
    r0, r1 = W.waveguide_rows(240, 0.025)
    assert (r0, r1) == (112, 128)
    assert np.all(g.eps[r0:r1, :x0] == np.float32(12.25))
    assert np.all(g.eps[:r0, :x0] == np.float32(2.085))
    region = g.eps[y0:y0 + wy, x0:x0 + wx]
    assert region.std() > 1.0                     # continuous design, not flat
    J = (g.b / (-1j * g.omega)).reshape(240, 480)
    cols = np.nonzero(np.abs(J).sum(0))[0]
    assert list(cols) == [30]
    assert abs(np.abs(J[:, 30]).max() - 1.0) < 1e-12
    # the mode is confined to the waveguide band
    assert np.abs(J[r0:r1, 30]).min() > 0.3 and np.abs(J[:60, 30]).max() < 1e-3
    assert np.array_equal(W.grating(1000).eps, g.eps)
    assert not np.array_equal(W.grating(1001).eps, g.eps)


def test_trajectory_steps_are_correlated_perturbations():
    tr = W.trajectory(3000, 300000, 4, 192, 96, 1.55)
    x0, y0, wx, wy = W.design_box(192, 96)
    regions = [t.eps[y0:y0 + wy, x0:x0 + wx].astype(np.float64) for t in tr]
    for a, b in zip(regions, regions[1:]):
        d = np.abs(b - a).max()
        assert 0 < d <= 0.05 * W.CONTRAST + 1e-5
    # outside the design region nothing changes
    mask = np.ones((96, 192), bool)
    mask[y0:y0 + wy, x0:x0 + wx] = False
    assert np.array_equal(tr[0].eps[mask], tr[-1].eps[mask])


def test_correlated_batch_layout():
    batch = W.correlated_batch(n_traj=3, steps=2)
    assert [b.nx for b in batch] == [192, 192, 320, 320, 480, 480]
    assert [b.wavelength for b in batch] == [1.30, 1.30, 1.55, 1.55, 1.30, 1.30]
