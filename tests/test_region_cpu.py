"""Irregular contours (Section 4.3): the enclosing circle and the region test.

Oracle pins use closed forms (square, equilateral and obtuse triangles, the
L-shaped region's area on a grid); the library's host functions (Welzl's
construction, even-odd rule) are compared with the oracle's brute-force
circle and winding number on random polygons.  No GPU is needed."""
import numpy as np
import pytest

import paper_1404_1768_amd as fm
import pencilgen as pg
from oracle import gfeast as o


def test_oracle_circle_closed_forms():
    sq = np.array([0, 2, 2 + 2j, 2j])
    c, r = o.enclosing_circle(sq)
    assert abs(c - (1 + 1j)) < 1e-12 and abs(r - np.sqrt(2)) < 1e-12
    eq = np.exp(2j * np.pi * np.arange(3) / 3) * 1.7 + 0.3j      # equilateral, circumradius 1.7
    c, r = o.enclosing_circle(eq)
    assert abs(c - 0.3j) < 1e-12 and abs(r - 1.7) < 1e-12
    ob = np.array([0, 4, 2 + 0.5j])                              # obtuse: the longest side's circle
    c, r = o.enclosing_circle(ob)
    assert abs(c - 2) < 1e-12 and abs(r - 2) < 1e-12
    c, r = o.enclosing_circle(sq, margin=0.25)
    assert abs(r - 1.25 * np.sqrt(2)) < 1e-12


def test_oracle_region_area_of_the_L():
    # cell centres of a 200 x 200 grid over [-1, 1]^2: exactly 3/4 lie in the L
    g = (np.arange(200) + 0.5) / 100 - 1
    X, Y = np.meshgrid(g, g)
    inside = o.inside_region((X + 1j * Y).ravel(), pg.L_REGION)
    assert inside.sum() == 30000
    # orientation does not matter
    assert np.array_equal(inside, o.inside_region((X + 1j * Y).ravel(), pg.L_REGION[::-1]))


def _star(rng, k):
    th = np.sort(rng.uniform(0, 2 * np.pi, k))
    rad = rng.uniform(0.3, 1.0, k)
    return rad * np.exp(1j * th) + complex(*rng.normal(size=2))


@pytest.mark.parametrize("seed", range(6))
def test_library_matches_oracle_on_random_polygons(seed):
    rng = np.random.default_rng(seed)
    v = _star(rng, 5 + seed)
    c, r = fm.enclosing_circle(v, margin=0.0)
    co, ro = o.enclosing_circle(v)
    assert abs(r - ro) < 1e-12 * max(1, ro) and abs(c - co) < 1e-10
    assert np.all(np.abs(v - c) <= r * (1 + 1e-12))
    pts = rng.uniform(-2, 2, 4000) + 1j * rng.uniform(-2, 2, 4000) + v.mean()
    got = fm.region_inside(v, pts)
    ref = o.inside_region(pts, v)
    # points within 1e-9 of an edge may be classified either way
    e0, e1 = v, np.roll(v, -1)
    t = np.clip(np.real((pts[:, None] - e0) * np.conj(e1 - e0)) / np.abs(e1 - e0) ** 2, 0, 1)
    dist = np.min(np.abs(pts[:, None] - (e0 + t * (e1 - e0))), axis=1)
    far = dist > 1e-9
    assert np.array_equal(got[far], ref[far])
    assert got.any() and (~got).any()


def test_library_region_arguments():
    with pytest.raises(fm.FeastError):
        fm.enclosing_circle(np.array([]), 0.1)
    with pytest.raises(fm.FeastError):
        fm.enclosing_circle(pg.L_REGION, -0.5)
    with pytest.raises(fm.FeastError):
        fm.region_inside(pg.L_REGION[:2], [0.0])
    c, r = fm.enclosing_circle(pg.L_REGION, 0.1)
    assert abs(c) < 1e-15 and abs(r - 1.1 * np.sqrt(2)) < 1e-12
