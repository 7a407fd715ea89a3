"""Seeded synthetic inputs: reproducible, with the stated statistics."""
import math

import numpy as np

import workloads as W


def test_grf_unit_variance_and_correlation_length():
    g = W.gaussian_random_field((48, 48, 48), 0.1, seed=3)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.0) < 1e-12
    # Gaussian-filtered white noise has correlation exp(-r^2 / (4 l^2)) at lag r
    lag = 5  # cells of 1/48
    r = lag / 48.0
    corr = np.mean(g * np.roll(g, lag, axis=2))
    assert abs(corr - math.exp(-r * r / (4 * 0.01))) < 0.08
    assert np.array_equal(g, W.gaussian_random_field((48, 48, 48), 0.1, seed=3))


def test_media_ranges_and_omega():
    c = W.grf_medium(32, seed=0)
    assert c.min() >= 1.0 and c.max() <= 4.5
    lay = W.layered_medium(64, seed=1)
    assert lay.min() >= 1.0 and lay.max() <= 5.0
    assert W.omega_for_ppw(1.0, 32, 10.0) == 2 * math.pi * 32 / 10.0
    wl = W.config_layered_256(n=64, nrhs=3)
    assert len(wl.rhs) == 3 and all(abs(f).sum() == 1.0 for f in wl.rhs)
    for (z, y, x) in wl.meta["sources"]:
        assert min(z, y, x) > wl.damp_cells and max(z, y, x) < 64 - wl.damp_cells - 1


def test_uneven_batch_sizes():
    inst = W.config_uneven_batch(count=6, seed=2, sizes=(8, 12))
    assert {w.n for w in inst} <= {8, 12}
    assert all(6.0 <= w.meta["ppw"] <= 12.0 for w in inst)
