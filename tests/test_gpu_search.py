"""Search (Algorithm 4) on the GPU: the same decisions as the oracle's Search
on the same random pool (trace estimate s_0, number of rank tests, columns
used, numerical rank t) and the same subspace; then Algorithm 5 from Search's
basis on the plan's cached factors, checked against the planted spectrum."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_1404_1768_amd as fm  # noqa: E402
import pencilgen as pg  # noqa: E402
from oracle import gfeast as o  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(*xs):
    return [torch.from_numpy(np.ascontiguousarray(x)).to(DEV) for x in xs]


def _case(seed):
    p = pg.make_pencil(240, m=40, inside=18, inside_radius=0.8, outside_r=(2.0, 8.0),
                       center=0.2 + 0.1j, radius=1.0, nodes=16, c=0.05, seed=200 + seed,
                       name="search-%d" % seed)
    pool = np.random.default_rng(300 + seed).normal(size=(p.n, 120)).astype(np.complex128)
    return p, pool


def _cosines(U, V):
    Qv, _ = np.linalg.qr(V)
    return np.linalg.svd(U.conj().T @ Qv, compute_uv=False)


@pytest.mark.parametrize("seed,pc,rounds", [(0, 3, 2), (4, 3, 1), (1, 5, 2)])
@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
def test_search_matches_oracle(seed, pc, rounds, prec):
    p, pool = _case(seed)
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    ref = o.search(o.ShiftedSolver(p.A, p.B, z), w, pool, p=pc, alpha=1.5)
    assert ref.rounds == rounds
    A, B, Y = to_dev(p.A, p.B, pool)
    with fm.Plan(p.n, 40, p.center, p.radius, p.nodes, prec=prec) as plan:
        U1, info = plan.search(A, B, Y, pc, alpha=1.5)
    U1 = U1.cpu().numpy()
    assert info["t"] == ref.t == p.s
    if prec == fm.FP64:
        assert (info["s0"], info["rounds"], info["used"]) == (ref.s0, ref.rounds, ref.used)
    else:  # complex64 solves: the trace can round to the neighbouring integer
        assert abs(info["s0"] - ref.s0) <= 1
    assert info["filters"] == ref.filters
    assert np.linalg.norm(U1.conj().T @ U1 - np.eye(info["t"])) < 1e-12
    assert _cosines(U1, ref.U1).min() > 1 - 1e-9
    # the planted eigenspace, up to the filter's outside values 1/(1 + mu^16) <= 1.5e-5
    # (angles near 1e-4 in the one-round cases)
    X_in = np.linalg.solve(p.Q, np.eye(p.n)[:, p.inside_mask])
    assert _cosines(U1, X_in).min() > 1 - (1e-7 if prec == fm.FP64 else 1e-5)


@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
def test_search_then_solve_from_finds_the_planted_spectrum(prec):
    p, pool = _case(2)
    A, B, Y = to_dev(p.A, p.B, pool)
    with fm.Plan(p.n, 40, p.center, p.radius, p.nodes, prec=prec, eps=1e-10) as plan:
        U1, info = plan.search(A, B, Y, 3)
        plan.set_m(info["t"])
        r = plan.solve_from(A, B, U1)
    assert r.flag == 1 and r.err <= 1e-10
    got = np.sort_complex(r.lam)
    ref = np.sort_complex(p.d[p.inside_mask])
    assert len(got) == len(ref) == info["t"]
    assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.abs(ref).max())
    # the whole of Algorithm 5 in the oracle from the oracle's own Search
    res, sr = o.gfeast_search(p.A, p.B, pool, p.center, p.radius, p.nodes, p=3)
    assert sr.t == info["t"] and np.max(np.abs(np.sort_complex(res.lam) - got)) < 1e-10


def test_search_reports_pool_exhaustion_and_full_rank_at_m():
    p, pool = _case(0)
    A, B, Y = to_dev(p.A, p.B, pool)
    with fm.Plan(p.n, 40, p.center, p.radius, p.nodes) as plan:
        with pytest.raises(fm.FeastError) as e:
            plan.search(A, B, Y[:, :10].contiguous(), 3)
        assert e.value.code == fm.FEAST_EINVAL and "exhausted" in plan.last_error()
    with fm.Plan(p.n, 12, p.center, p.radius, p.nodes) as plan:   # m below s = 18
        with pytest.raises(fm.FeastError) as e:
            plan.search(A, B, Y, 3)
        assert e.value.code == fm.FEAST_EINVAL and "full rank" in plan.last_error()


def test_search_full_size_workload():
    """Workload 2 at full size (n = 4000, N = 32, s = 100), the paper's p = 50
    and alpha = 1.5: t = s (outside eigenvalues at |mu| >= 1.3 have filter
    values below 2.2e-4 < tau), U_1 spans the planted eigenspace."""
    p = pg.workload(2)
    pool = np.random.default_rng(7).normal(size=(p.n, 400)).astype(np.complex128)
    A, B, Y = to_dev(p.A, p.B, pool)
    with fm.Plan(p.n, 240, p.center, p.radius, p.nodes, prec=fm.MIXED) as plan:
        U1, info = plan.search(A, B, Y, 50, alpha=1.5)
        assert info["t"] == p.s == 100
        plan.set_m(info["t"])
        r = plan.solve_from(A, B, U1)
    assert r.flag == 1 and len(r.lam) == 100 and r.err <= 1e-10
    d_in = np.sort_complex(p.d[p.inside_mask])
    assert np.max(np.abs(np.sort_complex(r.lam) - d_in)) <= 1e-10 * np.abs(d_in).max()
