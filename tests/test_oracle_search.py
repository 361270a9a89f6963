"""Pins of the oracle's Search (Algorithm 4, Section 4.1).

For the generated pencils ``A = P D Q``, ``B = P Q`` the spectral projector onto
the eigenvectors inside the circle is ``Pi = Q^{-1} diag(inside) Q`` (the
resolvent ``(zB - A)^{-1} B = Q^{-1} (zI - D)^{-1} Q`` integrated over the
circle), so the count ``s``, the eigenspace and the trace identity of
eq. (trace) are known in closed form.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import pencilgen as pg
from oracle import gfeast as o


def _pencil(n=160, inside=12, outside_r=(4.0, 10.0), cluster=0, seed=5):
    return pg.make_pencil(n, m=40, inside=inside, inside_radius=0.8, outside_r=outside_r,
                          center=0.3 - 0.2j, radius=1.0, nodes=32, c=0.05, cluster=cluster,
                          cluster_r=(1.05, 1.2), seed=seed, name="search")


def _projector(p):
    return np.linalg.solve(p.Q, p.inside_mask[:, None] * p.Q)


def _pool(n, cols, seed):
    # N(0,1) entries (the paper's Y is real), stored as complex
    return np.random.default_rng(seed).normal(size=(n, cols)).astype(np.complex128)


def _principal_cosines(U, X):
    Qx, _ = np.linalg.qr(X)
    return np.linalg.svd(U.conj().T @ Qx, compute_uv=False)


def test_trace_of_projector_is_count_and_estimator_mean():
    # eq. (trace): trace(Pi) = s, and E[trace(Y^* Pi Y)] / p = s for Gaussian Y
    p = _pencil()
    Pi = _projector(p)
    assert abs(np.trace(Pi) - p.s) < 1e-9
    rng = np.random.default_rng(11)
    pc, draws = 8, 600
    est = []
    for _ in range(draws):
        Y = rng.normal(size=(p.n, pc))
        est.append(np.real(np.trace(Y.T @ Pi @ Y)) / pc)
    est = np.array(est)
    se = est.std() / np.sqrt(draws)
    assert abs(est.mean() - p.s) < 4 * se
    # the oracle's s_0 (a ceiling of the same ratio) over the same kind of draws
    s0 = [o.trace_estimate(Y, Pi @ Y) for Y in (rng.normal(size=(p.n, pc)) for _ in range(200))]
    assert abs(np.mean(s0) - (p.s + 0.5)) < 1.0


def test_search_grows_to_the_count_and_the_eigenspace(monkeypatch):
    # outside eigenvalues at |mu| >= 4: the discrete filter 1/(1 + mu^32) leaves
    # them below 1e-19, so the numerical rank of the filtered block is s.  The
    # trace estimate is forced low so that the widening step has to grow the block
    # (4 -> 6 -> 9 -> 14 columns) to reach it.
    p = _pencil()
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    solver = o.ShiftedSolver(p.A, p.B, z)
    monkeypatch.setattr(o, "trace_estimate", lambda Y0, U: 1)
    sr = o.search(solver, w, _pool(p.n, 200, 1), p=4, alpha=1.5)
    assert (sr.t, sr.s0, sr.rounds, sr.used) == (12, 1, 4, 4 + 2 + 3 + 5)
    assert np.linalg.norm(sr.U1.conj().T @ sr.U1 - np.eye(sr.t)) < 1e-12
    X_in = np.linalg.solve(p.Q, np.eye(p.n)[:, p.inside_mask])   # eigenvectors inside
    assert _principal_cosines(sr.U1, X_in).min() > 1 - 1e-10


def test_search_from_the_trace_estimate():
    # with the trace estimate itself (s_0 close to s) one widening suffices
    p = _pencil()
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    solver = o.ShiftedSolver(p.A, p.B, z)
    sr = o.search(solver, w, _pool(p.n, 200, 1), p=4, alpha=1.5)
    assert sr.t == 12 and abs(sr.s0 - 12) <= 4 and sr.rounds <= 2


def test_search_one_round_when_the_start_block_is_wide_enough():
    p = _pencil()
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    solver = o.ShiftedSolver(p.A, p.B, z)
    sr = o.search(solver, w, _pool(p.n, 40, 2), p=20)
    assert (sr.t, sr.rounds, sr.used) == (12, 1, 20)
    assert abs(sr.s0 - 12) <= 4


def test_search_rank_is_relative_to_the_block_scale():
    # within a round, |R_ii| >= tau |R_11| does not change when Y is scaled
    # (one round: p >= s, so the first rank test stops)
    p = _pencil()
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    solver = o.ShiftedSolver(p.A, p.B, z)
    a = o.search(solver, w, _pool(p.n, 100, 3), p=20)
    b = o.search(solver, w, 1e-7 * _pool(p.n, 100, 3), p=20)
    assert a.t == b.t == p.s and a.rounds == b.rounds == 1


def test_search_counts_eigenvalues_just_outside_as_an_upper_bound():
    # a cluster at |mu| in [1.05, 1.2] keeps filter values 3e-3..0.2 > tau: Search
    # returns an upper bound s <= t <= s + cluster, as Algorithm 5 needs
    p = _pencil(n=200, inside=10, cluster=25)
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    solver = o.ShiftedSolver(p.A, p.B, z)
    sr = o.search(solver, w, _pool(p.n, 200, 4), p=8)
    assert p.s <= sr.t <= p.s + 25
    X_in = np.linalg.solve(p.Q, np.eye(p.n)[:, p.inside_mask])
    assert _principal_cosines(sr.U1, X_in).min() > 1 - 1e-8


def test_search_errors():
    p = _pencil()
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    solver = o.ShiftedSolver(p.A, p.B, z)
    with pytest.raises(ValueError, match="exhausted"):
        o.search(solver, w, _pool(p.n, 8, 5), p=4)
    with pytest.raises(ValueError, match="cap"):
        o.search(solver, w, _pool(p.n, 100, 5), p=4, t_max=8)


def test_gfeast_after_search_finds_the_planted_spectrum():
    p = _pencil()
    res, sr = o.gfeast_search(p.A, p.B, _pool(p.n, 200, 6), p.center, p.radius, p.nodes, p=4)
    assert res.flag == 1 and sr.t == 12
    got = np.sort_complex(res.lam)
    ref = np.sort_complex(p.d[p.inside_mask])
    assert len(got) == len(ref) and np.max(np.abs(got - ref)) < 1e-10


def test_planted_absolute_rank_threshold_is_caught(monkeypatch):
    # a rank test with an absolute threshold would change with the scale of Y
    p = _pencil()
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    solver = o.ShiftedSolver(p.A, p.B, z)

    def absolute_rank(R, tau):
        return int(np.count_nonzero(np.abs(np.diag(R)) >= tau))

    monkeypatch.setattr(o, "numerical_rank", absolute_rank)
    with pytest.raises((AssertionError, ValueError)):
        b = o.search(solver, w, 1e-7 * _pool(p.n, 100, 3), p=20)
        assert b.t == p.s
