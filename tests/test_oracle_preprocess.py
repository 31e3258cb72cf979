"""Pins of the pre-processing oracle (Sect. 3.2): star mask, NaN-aware
median, nearest sky, sigma-clipped bad pixel map and neighbour repair."""

import numpy as np

from oracle import preprocess as Q


def test_mask_disk_lattice_counts():
    cube = np.zeros((3, 16, 16), np.float32)
    out = Q.mask_disk(cube, [5.0, 8.0, 8.0], [7.0, 8.0, 8.0], np.array([0.0, 1.0, 2 ** 0.5]).tolist()[0])
    assert np.isnan(out[0]).sum() == 1 and np.isnan(out[0, 7, 5])
    out = Q.mask_disk(cube, [8.0] * 3, [8.0] * 3, 1.0)
    assert np.isnan(out[0]).sum() == 5                       # centre and its 4 neighbours
    out = Q.mask_disk(cube, [8.0] * 3, [8.0] * 3, 2 ** 0.5)
    assert np.isnan(out[1]).sum() == 9                       # the 3 x 3 square
    out = Q.mask_disk(cube, [8.5] * 3, [8.5] * 3, 0.75)
    assert np.isnan(out[2]).sum() == 4                       # the 4 pixels around a corner


def test_median_nan_brute_force():
    rng = np.random.default_rng(2)
    st = rng.normal(size=(9, 4, 5)).astype(np.float32)
    st[rng.random(st.shape) < 0.4] = np.nan
    st[:, 0, 0] = np.nan                                     # nothing left
    st[:, 1, 1] = np.nan
    st[4, 1, 1] = 3.5                                        # one value left
    got = Q.median_nan_f32(st)
    assert np.isnan(got[0, 0]) and got[1, 1] == np.float32(3.5)
    for y in range(4):
        for x in range(5):
            v = np.sort(st[:, y, x][~np.isnan(st[:, y, x])].astype(np.float64))
            if v.size:
                want = np.float32((v[(v.size - 1) // 2] + v[v.size // 2]) * 0.5)
                assert got[y, x] == want


def test_subtract_nearest_with_ties():
    cube = np.ones((4, 2, 2), np.float32) * 10
    skies = np.stack([np.full((2, 2), k, np.float32) for k in (1, 2, 3)])
    out = Q.subtract_nearest(cube, [0.0, 1.0, 4.9, 9.0], skies, [0.0, 2.0, 8.0])
    # 1.0 is equidistant from 0 and 2: the earlier sky wins
    assert out[:, 0, 0].tolist() == [9.0, 9.0, 8.0, 7.0]


def test_badpix_map_by_hand():
    f = np.zeros((4, 4), np.float32)
    f[1, 2] = 100.0
    f[3, 3] = np.nan
    # median 0, sigma over the 15 finite values = sqrt(100^2/15 - (100/15)^2)
    sigma = np.sqrt(100.0 ** 2 / 15 - (100.0 / 15) ** 2)
    bad = Q.badpix_map(f, 100.0 / sigma - 1e-9)
    assert bad.sum() == 2 and bad[1, 2] and bad[3, 3]
    assert Q.badpix_map(f, 100.0 / sigma + 1e-9).sum() == 1


def test_badpix_fix_restores_planes_and_clumps():
    yy, xx = np.mgrid[0:24, 0:24]
    plane = (3 * xx - 2 * yy + 50).astype(np.float32)[None]
    bad = np.zeros((24, 24), bool)
    bad[5, 7] = bad[12, 12] = bad[20, 3] = True                # isolated pixels
    out, passes = Q.badpix_fix(plane, bad)
    assert passes == 1
    assert np.array_equal(out, plane)        # the 8 neighbours of a plane pixel are symmetric about it
    flat = np.full((1, 24, 24), 7.25, np.float32)
    for k, want in ((3, 2), (5, 3)):         # a k x k clump fills from its rim inward
        bad = np.zeros((24, 24), bool)
        bad[8:8 + k, 9:9 + k] = True
        out, passes = Q.badpix_fix(flat, bad)
        assert passes == want and np.array_equal(out, flat)
    allnan = np.full((1, 4, 4), np.nan, np.float32)
    out, _ = Q.badpix_fix(allnan)
    assert np.isnan(out).all()
