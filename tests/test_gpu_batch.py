"""Batched form on the GPU: many pencils of uneven order whose shifted
systems are factored and solved in lockstep (grouped launches replayed from
HIP graphs), checked pencil by pencil

* against the oracle's filter and its Algorithm 5 run on the same inputs,
* against the spectrum the generator planted (A = P D Q, B = P Q: the
  eigenvalues inside each contour are the entries of D there),
* by residuals (eq. 5-1) recomputed on the host with the original A, B.

The small batches have orders that are not multiples of the 64-wide panel
(identity padding), equal orders (ties in the size ordering) and pencils that
stop at different iterations."""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_1404_1768_amd as fm  # noqa: E402
import pencilgen as pg  # noqa: E402
from oracle import gfeast as o  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def small_batch():
    ps = pg.batch_workload(count=6, lo=64, hi=300)
    # one more pencil with the order of the first (a tie) and an exact multiple of 64
    ps.append(pg.make_pencil(ps[0].n, m=ps[0].m, inside=ps[0].m // 2, inside_radius=0.9,
                             outside_r=(1.3, 10.0), center=-0.5 + 0.25j, radius=1.0, nodes=16,
                             c=0.05, seed=77, name="tie"))
    ps.append(pg.make_pencil(128, m=12, inside=6, inside_radius=0.9, outside_r=(1.3, 10.0),
                             center=1.0, radius=1.0, nodes=16, c=0.05, seed=78, name="n128"))
    # padded to 64: factored whole in LDS in either precision (128 and below in complex64)
    ps.append(pg.make_pencil(40, m=10, inside=4, inside_radius=0.8, outside_r=(1.3, 10.0),
                             center=0.3j, radius=1.0, nodes=16, c=0.05, seed=79, name="n40"))
    return ps


def make_batch(ps, prec=fm.FP64, **kw):
    return fm.Batch([p.n for p in ps], [p.m for p in ps], [p.center for p in ps],
                    [p.radius for p in ps], ps[0].nodes, prec=prec, **kw)


def host_residuals(A, B, lam, X):
    AX, BX = A @ X, B @ X
    return np.array([np.linalg.norm(AX[:, i] - lam[i] * BX[:, i]) /
                     (np.linalg.norm(AX[:, i]) + np.linalg.norm(BX[:, i])) for i in range(len(lam))])


def check_eigenvalues(lam, ref, radius):
    assert len(lam) == len(ref)
    C = np.abs(lam[:, None] - ref[None, :])
    ri, ci = linear_sum_assignment(C)
    scale = np.maximum(np.abs(ref[ci]), 1e-3 * radius)
    assert np.all(C[ri, ci] <= 1e-10 * scale), np.max(C[ri, ci] / scale)


@pytest.mark.parametrize("prec,sweeps", [(fm.FP64, 0), (fm.MIXED, 3)])
def test_batch_filter_matches_oracle(prec, sweeps):
    ps = small_batch()
    As, Bs, Vs = [to_dev(p.A) for p in ps], [to_dev(p.B) for p in ps], [to_dev(p.V) for p in ps]
    with make_batch(ps, prec) as b:
        Us = [u.cpu().numpy() for u in b.filter(As, Bs, Vs, sweeps)]
        # second call: cached factors, replayed graphs, the same blocks
        Us2 = [u.cpu().numpy() for u in b.filter(As, Bs, Vs, sweeps)]
    for p, U, U2 in zip(ps, Us, Us2):
        z, w = o.contour_nodes(p.center, p.radius, p.nodes)
        ref = o.apply_filter(o.ShiftedSolver(p.A, p.B, z), w, p.V)
        assert np.max(np.abs(U - ref)) <= 1e-10 * np.abs(ref).max(), p.name
        assert np.array_equal(U, U2), p.name


@pytest.mark.parametrize("prec,nb,upd", [(fm.FP64, 64, 1), (fm.FP64, 64, 2), (fm.FP64, 128, 1),
                                         (fm.FP64, 128, 3), (fm.MIXED, 64, 3), (fm.MIXED, 128, 1),
                                         (fm.MIXED, 128, 3)])
def test_batch_lu_configurations_match_oracle(prec, nb, upd):
    # every configuration the autotuner may pick (panel width, trailing-update
    # loop) gives the oracle's filtered blocks; orders 64..300 put odd multiples
    # of 64 (a last 64-column panel under 128-column steps) in the batch
    ps = small_batch()
    As, Bs, Vs = [to_dev(p.A) for p in ps], [to_dev(p.B) for p in ps], [to_dev(p.V) for p in ps]
    with make_batch(ps, prec, nb=nb, batch_update=upd) as b:
        Us = [u.cpu().numpy() for u in b.filter(As, Bs, Vs, 3 if prec == fm.MIXED else 0)]
    for p, U in zip(ps, Us):
        z, w = o.contour_nodes(p.center, p.radius, p.nodes)
        ref = o.apply_filter(o.ShiftedSolver(p.A, p.B, z), w, p.V)
        assert np.max(np.abs(U - ref)) <= 1e-10 * np.abs(ref).max(), (p.name, nb, upd)


def test_batch_filter_mixed_without_refinement_is_single_precision_accurate():
    ps = small_batch()[:3]
    As, Bs, Vs = [to_dev(p.A) for p in ps], [to_dev(p.B) for p in ps], [to_dev(p.V) for p in ps]
    with make_batch(ps, fm.MIXED) as b:
        U0 = [u.cpu().numpy() for u in b.filter(As, Bs, Vs, 0)]
        U1 = [u.cpu().numpy() for u in b.filter(As, Bs, Vs, 1)]
    for p, a, c in zip(ps, U0, U1):
        z, w = o.contour_nodes(p.center, p.radius, p.nodes)
        ref = o.apply_filter(o.ShiftedSolver(p.A, p.B, z), w, p.V)
        e0 = np.max(np.abs(a - ref)) / np.abs(ref).max()
        e1 = np.max(np.abs(c - ref)) / np.abs(ref).max()
        assert 1e-12 < e0 < 1e-4 and e1 < 1e-3 * e0, (e0, e1)


@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
def test_batch_solve_matches_oracle_and_planted_spectrum(prec):
    ps = small_batch()
    As, Bs, Vs = [to_dev(p.A) for p in ps], [to_dev(p.B) for p in ps], [to_dev(p.V) for p in ps]
    with make_batch(ps, prec, eps=1e-12, max_iter=20) as b:
        r = b.solve(As, Bs, Vs)
    assert r.info["graph_launches"] >= 2
    for i, p in enumerate(ps):
        assert r.flag[i] == 1, (p.name, r.flag[i], r.err[i])
        d_in = p.d[p.inside_mask]
        check_eigenvalues(r.lam[i], d_in, p.radius)
        ref = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-12, max_iter=20)
        check_eigenvalues(r.lam[i], ref.lam, p.radius)
        X = r.X[i].cpu().numpy()
        assert np.all(host_residuals(p.A, p.B, r.lam[i], X) <= 1e-10)
        assert np.all(r.res[i] <= 1e-10)


def test_batch_invalidate_refactors_changed_pencils():
    ps = small_batch()[:3]
    As, Bs, Vs = [to_dev(p.A) for p in ps], [to_dev(p.B) for p in ps], [to_dev(p.V) for p in ps]
    with make_batch(ps) as b:
        U = [u.cpu().numpy() for u in b.filter(As, Bs, Vs)]
        As[1].mul_(2.0)
        Bs[1].mul_(2.0)      # same pencil, same eigenvalues, different matrices
        b.invalidate()
        U2 = [u.cpu().numpy() for u in b.filter(As, Bs, Vs)]
    # (2B)^{-1}-type scaling: (z 2B - 2A)^{-1} 2B V = (zB - A)^{-1} B V
    for a, c, p in zip(U, U2, ps):
        assert np.max(np.abs(a - c)) <= 1e-11 * np.abs(a).max(), p.name


def test_batch_full_workload_counts_and_spectrum():
    """Workload 4 at full size (64 pencils, n in [256, 2048], N = 16, m = 2 floor(n/20)),
    FP64 and mixed, in the configuration the benchmark times: every pencil's
    count equals its planted inside count, eigenvalues match D to 1e-10
    relative, sampled residuals are recomputed on the host, and the two
    smallest pencils are compared with the oracle."""
    ps = pg.batch_workload()
    As, Bs, Vs = [to_dev(p.A) for p in ps], [to_dev(p.B) for p in ps], [to_dev(p.V) for p in ps]
    order = np.argsort([p.n for p in ps])
    for prec in (fm.FP64, fm.MIXED):
        with make_batch(ps, prec, eps=1e-10) as b:
            r = b.solve(As, Bs, Vs)
        for i, p in enumerate(ps):
            assert r.flag[i] == 1, (p.name, r.flag[i], r.err[i])
            assert r.err[i] <= 1e-10
            check_eigenvalues(r.lam[i], p.d[p.inside_mask], p.radius)
        for i in (order[0], order[len(ps) // 2], order[-1]):
            p = ps[i]
            X = r.X[i].cpu().numpy()
            assert np.all(host_residuals(p.A, p.B, r.lam[i], X) <= 1e-10), p.name
        for i in order[:2]:
            p = ps[i]
            ref = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-10, max_iter=20)
            check_eigenvalues(r.lam[i], ref.lam, p.radius)


@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
def test_batch_single_iteration_stops_every_pencil_at_the_iteration_cap(prec):
    """max_iter = 1: every pencil stops at k = 1 by the iteration cap (flag -1) while the
    second filter, launched ahead of the host eigensolves, is still in flight;
    the first iteration's Ritz pairs match the oracle's."""
    ps = small_batch()[:4]
    As, Bs, Vs = [to_dev(p.A) for p in ps], [to_dev(p.B) for p in ps], [to_dev(p.V) for p in ps]
    with make_batch(ps, prec, max_iter=1) as b:
        r = b.solve(As, Bs, Vs)
        r2 = b.solve(As, Bs, Vs)  # the batch is reusable after the filter left in flight
    for i, p in enumerate(ps):
        assert r.flag[i] == -1 and r2.flag[i] == -1
        ref = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, max_iter=1)
        assert ref.flag == -1
        assert len(r.lam[i]) == len(ref.lam) == len(r2.lam[i])
        tol = 1e-9 if prec == fm.FP64 else 1e-4  # (one unrefined complex64 filter)
        C = np.abs(r.lam[i][:, None] - ref.lam[None, :])
        ri, ci = linear_sum_assignment(C)
        assert np.max(C[ri, ci]) <= tol * max(1.0, abs(p.center) + p.radius)
        assert np.allclose(np.sort_complex(r.lam[i]), np.sort_complex(r2.lam[i]), rtol=0, atol=1e-12)
