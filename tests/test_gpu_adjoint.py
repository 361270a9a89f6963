"""Adjoint form on the GPU: left eigenvectors from the adjoint filter on the
forward LU factors, and gradients of L = sum |lambda_i|^2 over the eigenvalues
inside the contour, checked against

* the closed form of the generated pencils (x_i = Q^{-1} e_i, y_i = P^{-*} e_i,
  y_i^* B x_i = 1, so dL/dA = 2 P^{-*} Lambda_in Q^{-*}, dL/dB = -2 P^{-*} |Lambda_in|^2 Q^{-*}),
* the oracle's gradient (brute-force left/right eigenvectors at small n; the
  oracle's Algorithm 5 and adjoint-filter left eigenvectors at n = 2048),
* the analytic eigenvalue derivatives y^*(dA - lambda dB) x / (y^* B x) of the
  oracle's eigenpairs, direction by direction,
* central finite differences of the GPU path (h = 1e-7).

Acceptance: gradients within 1e-6 relative."""
import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_1404_1768_amd as fm  # noqa: E402
import pencilgen as pg  # noqa: E402
from oracle import gfeast as o  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in arrs]


def closed_form_grads(p):
    Qi, Pi = np.linalg.inv(p.Q), np.linalg.inv(p.P)
    lam_in = np.where(p.inside_mask, p.d, 0)
    GA = 2.0 * Pi.conj().T @ np.diag(lam_in) @ Qi.conj().T
    GB = -2.0 * Pi.conj().T @ np.diag(np.abs(lam_in) ** 2) @ Qi.conj().T
    return GA, GB


def run_grad(p, sweeps=3):
    A, B, V = to_dev(p.A, p.B, p.V)
    A.requires_grad_(True)
    B.requires_grad_(True)
    with fm.Plan(p.n, p.m, p.center, p.radius, p.nodes, eps=1e-14, max_iter=8) as plan:
        lam = fm.feast_eig(A, B, V, plan, sweeps)
        loss = (lam.abs() ** 2).sum()
        loss.backward()
    return lam.detach().cpu().numpy(), A.grad.cpu().numpy(), B.grad.cpu().numpy()


def test_left_eigvecs_properties():
    p = pg.workload(5, n_override=512)
    A, B, V = to_dev(p.A, p.B, p.V)
    with fm.Plan(p.n, p.m, p.center, p.radius, p.nodes, eps=1e-13) as plan:
        r = plan.solve(A, B, V)
        Y = plan.left_eigvecs(A, B, r.X, 3).cpu().numpy()
    X = r.X.cpu().numpy()
    assert len(r.lam) == p.s
    # closed form: x = Q^{-1} e_k alpha  =>  y = P^{-*} e_k / conj(alpha)
    QX, Pi_h = p.Q @ X, np.linalg.inv(p.P).conj().T
    Yc = np.stack([Pi_h[:, np.argmax(np.abs(QX[:, i]))] / np.conj(QX[np.argmax(np.abs(QX[:, i])), i])
                   for i in range(p.s)], axis=1)
    assert np.linalg.norm(Y - Yc) / np.linalg.norm(Yc) < 1e-11
    # biorthonormal: Y^* B X = I and Y^* A X = diag(lambda)
    assert np.max(np.abs(Y.conj().T @ p.B @ X - np.eye(p.s))) < 1e-10
    assert np.max(np.abs(Y.conj().T @ p.A @ X - np.diag(r.lam))) < 1e-10
    # each y_i is a left eigenvector: (A - lambda_i B)^* y_i = 0
    for i in range(p.s):
        res = np.linalg.norm((p.A - r.lam[i] * p.B).conj().T @ Y[:, i])
        assert res <= 1e-10 * (np.linalg.norm(p.A) + abs(r.lam[i]) * np.linalg.norm(p.B)) * np.linalg.norm(Y[:, i])


_ORACLE = {}


def oracle_pairs(p):
    """The oracle's eigenpairs inside the contour with their left eigenvectors:
    brute-force QZ for small n; at the differentiation workload's n = 2048 the
    oracle's own Algorithm 5 and its adjoint-filter left eigenvectors (both
    pinned on the CPU), cached per order."""
    if p.n not in _ORACLE:
        if p.n <= 512:
            ev, Yl, Xr = sla.eig(p.A, p.B, left=True, right=True)
            sel = np.abs(ev - p.center) < p.radius
            _ORACLE[p.n] = (ev[sel], Xr[:, sel], Yl[:, sel])
        else:
            z, w = o.contour_nodes(p.center, p.radius, p.nodes)
            S = o.ShiftedSolver(p.A, p.B, z)
            r = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-13, solver=S)
            assert r.flag == 1 and len(r.lam) == p.s
            _ORACLE[p.n] = (r.lam, r.X, o.left_eigenvectors(S, w, p.B, r.X, 3))
    return _ORACLE[p.n]


def analytic_directional(p, dA, dB):
    """dL along (dA, dB) for L = sum |lambda_i|^2 from the oracle's eigenvalue
    derivatives y_i^*(dA - lambda_i dB) x_i / (y_i^* B x_i): sum 2 Re(conj(lambda_i) d lambda_i)."""
    lam, X, Yl = oracle_pairs(p)
    dl = o.eigenvalue_derivatives(p.B, lam, X, Yl, dA, dB)
    return float(np.sum(2.0 * np.real(np.conj(lam) * dl)))


@pytest.mark.parametrize("n", [256, 2048])
def test_gradient_matches_closed_form_and_oracle(n):
    p = pg.workload(5, n_override=n if n != 2048 else None)
    lam, GA, GB = run_grad(p)
    GAc, GBc = closed_form_grads(p)
    assert np.linalg.norm(GA - GAc) / np.linalg.norm(GAc) < 1e-8
    assert np.linalg.norm(GB - GBc) / np.linalg.norm(GBc) < 1e-8
    lo, Xo, Yo = oracle_pairs(p)
    GAo, GBo = o.loss_gradient(p.B, lo, Xo, Yo)
    assert np.linalg.norm(GA - GAo) / np.linalg.norm(GAo) < 1e-8
    assert np.linalg.norm(GB - GBo) / np.linalg.norm(GBo) < 1e-8


@pytest.mark.parametrize("n,ndir", [(512, 8), (2048, 32)])
def test_gradient_finite_differences(n, ndir):
    """Directional derivatives Re<G_A, dA> + Re<G_B, dB> of the GPU gradient
    against central differences of the GPU path (h = 1e-7) and against the
    analytic eigenvalue derivatives y_i^*(dA - lambda_i dB) x_i / (y_i^* B x_i)
    of the oracle's eigenpairs (n = 2048: the differentiation workload, 32
    directions).

    Directions with an O(1) derivative -- the normalised gradient, and the
    rank-one y_k x_k^* in A and in B for several k -- are checked relative to
    their own derivative (1e-6 against the differences, 1e-8 against the
    analytic value).  A random unit direction has a derivative of about
    ||grad L|| / n, below the differences' noise (about 1e-7 absolute: the
    forward solves are converged to rounding), so there the differences are
    checked relative to ||grad L|| and the analytic value per direction."""
    p = pg.workload(5, n_override=n if n != 2048 else None)
    lam, GA, GB = run_grad(p)
    A, B, V = to_dev(p.A, p.B, p.V)
    h = 1e-7
    rng = np.random.default_rng(21)
    lo, Xo, Yo = oracle_pairs(p)
    with fm.Plan(p.n, p.m, p.center, p.radius, p.nodes, eps=1e-14, max_iter=8) as plan:
        def loss(Ad, Bd):
            r = plan.solve(Ad, Bd, V)
            assert len(r.lam) == p.s
            return float(np.sum(np.abs(r.lam) ** 2))
        gnorm = np.sqrt(np.linalg.norm(GA) ** 2 + np.linalg.norm(GB) ** 2)
        dirs = [(GA / gnorm, GB / gnorm, True)]
        # rank-one directions in A (phase lambda_k/|lambda_k|) and in B (phase -1):
        # d lambda_k then makes conj(lambda_k) d lambda_k real positive, so the
        # k-th term 2 Re(conj(lambda_k) d lambda_k) is 2 |lambda_k| ||y_k|| ||x_k||
        # (A) or 2 |lambda_k|^2 ||y_k|| ||x_k|| (B), for the 4 largest |lambda_k|
        for k in np.argsort(-np.abs(lo))[:4]:
            R1 = np.outer(Yo[:, k], Xo[:, k].conj())
            R1 /= np.linalg.norm(R1)
            dirs.append((R1 * (lo[k] / abs(lo[k])), np.zeros_like(R1), True))
            dirs.append((np.zeros_like(R1), -R1, True))
        while len(dirs) < ndir:
            dA = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
            dB = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
            nr = np.sqrt(np.linalg.norm(dA) ** 2 + np.linalg.norm(dB) ** 2)
            dirs.append((dA / nr, dB / nr, False))
        worst = 0.0
        for dA, dB, order_one in dirs[:ndir]:
            tdA, tdB = to_dev(dA, dB)
            fd = (loss(A + h * tdA, B + h * tdB) - loss(A - h * tdA, B - h * tdB)) / (2 * h)
            an = np.real(np.vdot(GA, dA)) + np.real(np.vdot(GB, dB))
            ref = analytic_directional(p, dA, dB)
            assert abs(an - ref) <= 1e-8 * max(abs(ref), 1e-3 * gnorm), (an, ref)
            if order_one:
                assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
            worst = max(worst, abs(fd - an) / gnorm)
    assert worst < 1e-6, worst
