"""The seeded generator is deterministic and follows its stated recipe."""

import math

import numpy as np

import synth


def test_same_seed_same_cube():
    a = synth.render_host(synth.make_params(1, T=3, N=32))
    b = synth.render_host(synth.make_params(1, T=3, N=32))
    assert a.tobytes() == b.tobytes()
    c = synth.render_host(synth.make_params(1, T=3, N=32, seed=5))
    assert a.tobytes() != c.tobytes()


def test_recipe_shapes_and_ranges():
    p = synth.make_params(1)
    assert (p.T, p.N, p.P) == (16, 128, 256)
    assert np.all(np.abs(p.dx) <= 0.5) and np.all(np.abs(p.dy) <= 0.5)
    assert np.all(np.diff(p.parang) >= 0) and p.parang.min() >= 0 and p.parang.max() <= 30
    q = synth.make_params(2, T=8, N=64)
    assert np.allclose(q.parang, np.linspace(-30, 30, 8))
    assert np.all(np.abs(q.dx) <= 1.0)
    assert len(q.companions) == 3


def test_companion_follows_field_rotation():
    p = synth.make_params(1, T=4, N=64)
    for i in range(p.T):
        (x, y), = synth.companion_positions(p, i)
        ux, uy = x - (32 - p.dx[i]), y - (32 - p.dy[i])
        assert abs(math.hypot(ux, uy) - 20.0) < 1e-9
        assert abs(math.degrees(math.atan2(uy, ux)) - p.parang[i]) < 1e-9


def test_star_core_peak_and_halo_level():
    p = synth.make_params(1, T=1, N=128)
    f = synth.render_host(p)[0].astype(np.float64)
    yy, xx = np.mgrid[0:128, 0:128]
    r = np.hypot(xx - 64 + p.dx[0], yy - 64 + p.dy[0])
    ring = (r > 9.5) & (r < 10.5)
    assert 50 < f[ring].mean() < 200
    assert 0.8e4 < f.max() < 1.5e4


def test_batch_and_arrivals():
    b = synth.make_batch_params(n_cubes=6, with_screen=False)
    assert all(32 <= p.T <= 2048 and p.N in (256, 512, 1024, 2048) for p in b)
    t = synth.make_arrivals(100, 20.0)
    assert np.all(np.diff(t) > 0) and 2.0 < t[-1] < 10.0
