"""Algorithm 5 on the GPU through the C ABI, on the paths the method itself
takes:

* the benchmark configuration (n = 4000, N = 32, m = 160, complex64 LU with
  FP64 refinement, started from V) against the oracle's own Algorithm 5 run
  and the planted spectrum;
* the no-improvement rule (flag 0: iterate k-1 and Err = e(k-1) returned),
  single pencil and batched;
* factor reuse only for the pencil the factors belong to (Section 4.3): a
  different pencil at the same device address, and a pencil changed in place.

Acceptance (the method's targets): eigenvalues within 1e-10 relative of the
oracle and of the planted spectrum, eigenvectors with |x_gpu^* x_oracle| >=
1 - 1e-10, and every returned residual (eq. 5-1, recomputed on the host with
the original A and B) at most 1e-10.
"""
import warnings

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_1404_1768_amd as fm  # noqa: E402
import pencilgen as pg  # noqa: E402
from oracle import gfeast as o  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in arrs]


def match(lam, ref):
    C = np.abs(lam[:, None] - ref[None, :])
    ri, ci = linear_sum_assignment(C)
    return ri, ci, C[ri, ci]


def host_residuals(A, B, lam, X):
    AX, BX = A @ X, B @ X
    return np.array([np.linalg.norm(AX[:, i] - lam[i] * BX[:, i]) /
                     (np.linalg.norm(AX[:, i]) + np.linalg.norm(BX[:, i])) for i in range(len(lam))])


def test_benchmark_configuration_mixed_against_oracle():
    """n = 4000, N = 32, m = 160, MIXED, from the workload's V (the metric's
    configuration): count 100, eigenvalues against the planted spectrum and
    the oracle's Algorithm 5 (1e-10 relative), eigenvector overlaps with the
    oracle's, host residuals <= 1e-10."""
    p = pg.workload(2)
    A, B, V = to_dev(p.A, p.B, p.V)
    print("case: workload n=%d m=%d N=%d mixed" % (p.n, p.m, p.nodes), flush=True)
    with fm.Plan(p.n, p.m, p.center, p.radius, p.nodes, prec=fm.MIXED, eps=1e-10) as plan:
        r = plan.solve(A, B, V)
    X = r.X.cpu().numpy()
    del A, B, V
    assert r.flag == 1 and r.err <= 1e-10, (r.flag, r.err, r.errs)
    assert len(r.lam) == p.s == 100
    exact = p.d[p.inside_mask]
    _, ci, d = match(r.lam, exact)
    assert np.max(d / np.maximum(np.abs(exact[ci]), 1e-3 * p.radius)) <= 1e-10
    assert host_residuals(p.A, p.B, r.lam, X).max() <= 1e-10
    ref = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-10)
    assert ref.flag == 1 and len(ref.lam) == 100
    ri, ci, d = match(r.lam, ref.lam)
    assert np.max(d / np.maximum(np.abs(ref.lam[ci]), 1e-3 * p.radius)) <= 1e-10
    ov = np.abs(np.sum(np.conj(ref.X[:, ci]) * X[:, ri], axis=0))
    assert ov.min() >= 1 - 1e-10, ov.min()


def _check_rebound(lam, X, res, err, flag, errs, counts, A, B, ref):
    """The no-improvement stop of Algorithm 5: the last iteration kept the
    count and raised e(k); the returned pairs are iterate k-1's, Err = e(k-1).
    The iteration at which rounding-level errors first rise is decided by
    rounding on each side, so the oracle is compared on what is unique -- the
    converged eigenpairs -- and the rest is checked for validity."""
    k = len(errs)
    assert flag == 0, (flag, errs)
    assert k >= 2 and counts[-1] == counts[-2] and errs[-1] > errs[-2]
    assert err == errs[-2]
    assert len(lam) == counts[-2] == len(ref.lam)
    assert err == max(res)                               # Err = max r_i of iterate k-1
    hr = host_residuals(A, B, lam, X)
    assert hr.max() <= 1e-10
    assert np.allclose(hr, res, rtol=0.5, atol=1e-15)    # the returned residuals are these pairs'
    ri, ci, d = match(lam, ref.lam)
    assert np.max(d / np.maximum(np.abs(ref.lam[ci]), 1e-3)) <= 1e-10
    ov = np.abs(np.sum(np.conj(ref.X[:, ci]) * X[:, ri], axis=0))
    assert ov.min() >= 1 - 1e-10


@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
def test_no_improvement_rule_single(prec):
    """eps below the attainable floor: rule 13 cannot fire, so the run ends on
    rule 14 once e(k) rises at the rounding floor (the oracle's rebound
    setting, n = 200, 20 eigenvalues inside)."""
    p = pg.workload(1)
    ref = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-300, max_iter=40)
    assert ref.flag == 0
    A, B, V = to_dev(p.A, p.B, p.V)
    with fm.Plan(p.n, p.m, p.center, p.radius, p.nodes, prec=prec, eps=1e-300,
                 max_iter=40) as plan:
        r = plan.solve(A, B, V)
    _check_rebound(r.lam, r.X.cpu().numpy(), r.res, r.err, r.flag, r.errs, r.count, p.A, p.B, ref)


@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
def test_no_improvement_rule_batched(prec):
    """The same rule per pencil in the batched form (pencils stop at their own
    iterations while the others continue)."""
    ps = pg.batch_workload(count=4, lo=128, hi=400)
    refs = [o.gfeast(q.A, q.B, q.V, q.center, q.radius, q.nodes, eps=1e-300, max_iter=40)
            for q in ps]
    assert all(rf.flag == 0 for rf in refs)
    As, Bs, Vs = [to_dev(q.A)[0] for q in ps], [to_dev(q.B)[0] for q in ps], \
        [to_dev(q.V)[0] for q in ps]
    with fm.Batch([q.n for q in ps], [q.m for q in ps], [q.center for q in ps],
                  [q.radius for q in ps], ps[0].nodes, prec=prec, eps=1e-300, max_iter=40) as b:
        r = b.solve(As, Bs, Vs)
    for i, q in enumerate(ps):
        assert r.flag[i] == 0, (i, r.flag, r.iters)
        assert len(r.lam[i]) == q.s == len(refs[i].lam)
        assert r.err[i] == max(r.res[i])
        X = r.X[i].cpu().numpy()
        hr = host_residuals(q.A, q.B, r.lam[i], X)
        assert hr.max() <= 1e-10
        _, ci, d = match(r.lam[i], refs[i].lam)
        assert np.max(d / np.maximum(np.abs(refs[i].lam[ci]), 1e-3)) <= 1e-10


# ---------------------------------------------------------------------------
# Factor reuse belongs to the pencil (Section 4.3)
# ---------------------------------------------------------------------------

def _two_pencils(n=200):
    p1 = pg.workload(1)
    p2 = pg.make_pencil(n, m=p1.m, inside=14, inside_radius=0.8, outside_r=(1.5, 5.0),
                        center=p1.center, radius=p1.radius, nodes=p1.nodes, c=0.1, seed=404)
    return p1, p2


def _check_spectrum(r, p):
    assert r.flag == 1 and len(r.lam) == p.s
    exact = p.d[p.inside_mask]
    _, ci, d = match(r.lam, exact)
    assert np.max(d / np.maximum(np.abs(exact[ci]), 1e-3)) <= 1e-10


@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
def test_new_pencil_at_the_same_address_is_refactored(prec):
    """A freed pencil's memory handed to a new pencil of the same shape, as
    PyTorch's caching allocator does: new tensors over the same storage."""
    p1, p2 = _two_pencils()
    n = p1.n
    store = torch.empty(2 * n * n, dtype=torch.complex128, device=DEV)
    A, B = store[:n * n].view(n, n), store[n * n:].view(n, n)
    A.copy_(torch.from_numpy(p1.A))
    B.copy_(torch.from_numpy(p1.B))
    (V,) = to_dev(p1.V)
    with fm.Plan(p1.n, p1.m, p1.center, p1.radius, p1.nodes, prec=prec) as plan:
        _check_spectrum(plan.solve(A, B, V), p1)
        pa, pb = A.data_ptr(), B.data_ptr()
        del A, B
        A2, B2 = store[:n * n].view(n, n), store[n * n:].view(n, n)
        assert (A2.data_ptr(), B2.data_ptr()) == (pa, pb)
        A2.copy_(torch.from_numpy(p2.A))
        B2.copy_(torch.from_numpy(p2.B))
        _check_spectrum(plan.solve(A2, B2, V), p2)
        # and back in place: the first pencil again at the same addresses
        A2.copy_(torch.from_numpy(p1.A))
        B2.copy_(torch.from_numpy(p1.B))
        _check_spectrum(plan.solve(A2, B2, V), p1)


def test_in_place_change_of_A_refactors_filter_and_batch():
    """feast_filter after A changes in place equals the oracle's filter of the
    new pencil; the batched form likewise refactors a changed pencil."""
    p1, p2 = _two_pencils()
    A, B, V = to_dev(p1.A, p1.B, p1.V)
    with fm.Plan(p1.n, p1.m, p1.center, p1.radius, p1.nodes) as plan:
        plan.filter(A, B, V)
        A.copy_(torch.from_numpy(p2.A))
        B.copy_(torch.from_numpy(p2.B))
        U = plan.filter(A, B, V).cpu().numpy()
    z, w = o.contour_nodes(p2.center, p2.radius, p2.nodes)
    ref = o.apply_filter(o.ShiftedSolver(p2.A, p2.B, z), w, p1.V)
    assert np.max(np.abs(U - ref)) <= 1e-11 * np.abs(ref).max()
    # batch: pencil 1 of 2 changes in place between two solves
    A1, B1, V1 = to_dev(p1.A, p1.B, p1.V)
    A0, B0, V0 = to_dev(p1.A, p1.B, p1.V)
    with fm.Batch([p1.n, p1.n], [p1.m, p1.m], [p1.center] * 2, [p1.radius] * 2,
                  p1.nodes) as b:
        r = b.solve([A0, A1], [B0, B1], [V0, V1])
        assert all(len(x) == p1.s for x in r.lam)
        A1.copy_(torch.from_numpy(p2.A))
        B1.copy_(torch.from_numpy(p2.B))
        r = b.solve([A0, A1], [B0, B1], [V0, V1])
    assert len(r.lam[0]) == p1.s and len(r.lam[1]) == p2.s
    exact = p2.d[p2.inside_mask]
    _, ci, d = match(r.lam[1], exact)
    assert np.max(d / np.maximum(np.abs(exact[ci]), 1e-3)) <= 1e-10


def test_feast_eig_warns_when_not_converged():
    p = pg.workload(1)
    A, B, V = to_dev(p.A, p.B, p.V)
    with fm.Plan(p.n, p.m, p.center, p.radius, p.nodes, max_iter=1) as plan:
        with warnings.catch_warnings(record=True) as rec:
            warnings.simplefilter("always")
            lam = fm.feast_eig(A, B, V, plan)
    assert lam.shape[0] == p.s
    assert any(issubclass(x.category, RuntimeWarning) and "flag -1" in str(x.message) for x in rec)


# ---------------------------------------------------------------------------
# Badly scaled pencils
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [1e30, 1e-30])
@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
def test_scaled_pencil(scale, prec):
    """(s A, s B) has the eigenpairs of (A, B).  At s = 1e+-30 the complex64
    pivots' squared moduli leave complex64's range (the reciprocal must be
    scaled) and complex64 refinement residuals of order 1e-16 s would be
    subnormal (the solves are scaled by a power of two): both forms must still
    return the planted eigenvalues with residuals <= 1e-10."""
    p = pg.workload(1)
    A, B, V = to_dev(scale * p.A, scale * p.B, p.V)
    print("case: n=%d scale=%g prec=%d" % (p.n, scale, prec), flush=True)
    with fm.Plan(p.n, p.m, p.center, p.radius, p.nodes, prec=prec, eps=1e-10) as plan:
        r = plan.solve(A, B, V)
    _check_spectrum(r, p)
    assert r.err <= 1e-10
    X = r.X.cpu().numpy()
    assert host_residuals(p.A, p.B, r.lam, X).max() <= 1e-10
