"""Host side of the sparse path (no GPU): the ordering feast_solve_csr applies
to a pencil's pattern (reverse Cuthill-McKee, or the natural order where that
is as narrow), its refusal of malformed patterns, and the banded stand-ins of
Table 1 that the sparse GPU tests use."""
import json
import math
import os

import numpy as np
import pytest

import paper_1404_1768_amd as fm
import pencilgen as pg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "standin_banded_contours.json")


def _pattern(rows, cols, n):
    o = np.lexsort((cols, rows))
    rows, cols = np.asarray(rows)[o], np.asarray(cols)[o]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), cols.astype(np.int32)


def _band_pattern(n, bw, seed, density=0.6):
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        for j in range(max(0, i - bw), min(n, i + bw + 1)):
            if i == j or abs(i - j) == 1 or rng.random() < density:
                rows.append(i)
                cols.append(j)
    return np.array(rows), np.array(cols)


@pytest.mark.parametrize("n,bw,seed", [(300, 3, 0), (1000, 10, 1), (777, 22, 2)])
def test_rcm_recovers_a_scrambled_band(n, bw, seed):
    rows, cols = _band_pattern(n, bw, seed)
    q = np.random.default_rng(seed + 100).permutation(n)   # old index i -> new index q[i]
    rp, ci = _pattern(q[rows], q[cols], n)
    assert np.abs(q[rows] - q[cols]).max() > 10 * bw       # scrambled
    perm, kl, ku = fm.csr_order(rp, ci)
    assert sorted(perm.tolist()) == list(range(n))
    # the widths it reports are those of the reordered pattern
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    r2, c2 = inv[q[rows]], inv[q[cols]]
    assert kl == (r2 - c2).max() and ku == (c2 - r2).max()
    # a connected band (the sub/superdiagonals are kept) comes back within
    # twice its width (reverse Cuthill-McKee's level structure of a band)
    assert kl <= 2 * bw and ku <= 2 * bw
    # in its natural order the band is kept: reverse Cuthill-McKee is used
    # only where it is narrower
    rp0, ci0 = _pattern(rows, cols, n)
    perm0, kl0, ku0 = fm.csr_order(rp0, ci0)
    assert kl0 + ku0 <= 2 * bw


def test_rcm_components_and_isolated_vertices():
    # two bands and a set of isolated vertices, interleaved
    n = 90
    rows, cols = [], []
    for i in range(0, 40):
        for j in (i - 1, i, i + 1):
            if 0 <= j < 40:
                rows.append(2 * i)
                cols.append(2 * j)
    for i in range(40, 45):
        rows.append(2 * i - 79)
        cols.append(2 * i - 79)
    rp, ci = _pattern(np.array(rows), np.array(cols), n)
    perm, kl, ku = fm.csr_order(rp, ci)
    assert sorted(perm.tolist()) == list(range(n))
    assert kl <= 2 and ku <= 2


def test_rcm_rejects_malformed_patterns():
    rp = np.array([0, 2, 3], np.int32)
    with pytest.raises(fm.FeastError):
        fm.csr_order(rp, np.array([0, 0, 1], np.int32))          # column twice in a row
    with pytest.raises(fm.FeastError):
        fm.csr_order(rp, np.array([0, 2, 1], np.int32))          # column out of range
    with pytest.raises(fm.FeastError):
        fm.csr_order(np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32))  # decreasing


@pytest.mark.parametrize("k", range(1, 8))
def test_banded_standins_shape(k):
    name, A, B, V = pg.sparse_standin(k, banded=True)
    n, nnz_a, nnz_b = pg.TABLE1[k - 1][1:4]
    band = math.ceil(nnz_a / n)
    assert A.shape == (n, n) and V.shape == (n, 40)
    for M, nnz in ((A, nnz_a), (B, nnz_b)):
        i, j = np.nonzero(M)
        assert np.abs(i - j).max() <= band
        # collisions of the random positions remove a few per cent of the entries
        assert 0.8 * nnz <= i.size <= 1.02 * nnz
    # the sparse path accepts it: bandwidths of the union pattern
    Sa = np.abs(A) + np.abs(B)
    r, c = np.nonzero(Sa)
    rp, ci = _pattern(r, c, n)
    perm, kl, ku = fm.csr_order(rp, ci)
    assert kl + ku <= 63


def test_banded_golden_contours():
    with open(GOLDEN) as f:
        g = json.load(f)
    assert sorted(g, key=int) == [str(k) for k in range(1, 8)]
    for k, e in g.items():
        assert e["n"] == pg.TABLE1[int(k) - 1][1]
        assert 1 <= e["s"] <= 20 and len(e["inside"]) == e["s"]
        c = complex(*e["center"])
        assert all(abs(complex(*z) - c) < e["radius"] for z in e["inside"])
        assert e["gap"] > 1.1
