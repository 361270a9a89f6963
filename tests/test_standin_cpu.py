"""Sparse-shaped stand-ins of Table 1 (Section 5): the generated pencils have
the orders, numbers of non-zeros and structure the table lists, and the stored
contours (tests/golden/standin_contours.json, written by the oracle only)
reproduce from the oracle's dense reference spectrum."""
import json
import os

import numpy as np
import pytest

import pencilgen as pg
from oracle import gfeast as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "standin_contours.json")


def _load():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_standin_shapes_match_table1(k):
    name, n, nnz_a, nnz_b, ka, kb = pg.TABLE1[k - 1]
    nm, A, B, V = pg.sparse_standin(k)
    assert nm == name and A.shape == B.shape == (n, n) and V.shape == (n, 40)
    assert np.all(A.imag == 0) and np.all(B.imag == 0)
    for M, nnz, kind in ((A.real, nnz_a, ka), (B.real, nnz_b, kb)):
        # random patterns collide a little: within 10% of the table's count
        assert abs(np.count_nonzero(M) - nnz) <= 0.1 * nnz
        if kind in ("symind", "spd", "spsd"):
            assert np.array_equal(M, M.T)
        if kind == "skew":
            assert np.array_equal(M, -M.T)
        if kind == "spd":
            assert np.linalg.eigvalsh(M).min() > 0
        if kind == "unsym":
            assert not np.array_equal(M, M.T)


def test_fixture_covers_table1():
    g = _load()
    assert sorted(g, key=int) == [str(k) for k in range(1, 8)]
    for k, e in g.items():
        name, n = pg.TABLE1[int(k) - 1][:2]
        assert e["name"] == name and e["n"] == n
        assert len(e["inside"]) == e["s"] and 8 <= e["s"] <= 28
        c = complex(*e["center"])
        d = np.abs(np.array([complex(*z) for z in e["inside"]]) - c)
        assert np.all(d < e["radius"])
        assert e["gap"] > 1.0


def test_fixture_reproduces_from_the_oracle():
    g = _load()["1"]
    _, A, B, _ = pg.sparse_standin(1)
    lam = o.dense_eigenvalues(A, B)
    c, r, s, gap = o.standin_contour(lam)
    assert s == g["s"] and abs(c - complex(*g["center"])) < 1e-12 and abs(r - g["radius"]) < 1e-12
    ref = np.array([complex(*z) for z in g["inside"]])
    got = lam[np.abs(lam - c) < r]
    assert got.size == ref.size
    assert np.max(np.min(np.abs(got[:, None] - ref[None, :]), axis=1)) < 1e-10
