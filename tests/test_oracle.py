"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
formula: they check printed values (Example 3.1), closed forms derived from the
Weierstrass form of the generated pencils, identities, brute-force
eigendecompositions and planted mistakes.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import pencilgen as pg
from oracle import gfeast as o
from conftest import load_example31


def _closed_form_filter(p, z, w, V):
    """``Q_N V = Q^{-1} f(D) Q V`` for ``A = P D Q``, ``B = P Q``: the resolvent of
    eq. (8-3-4) with ``S = Q^{-1}``, ``T = P^{-1}`` is ``Q^{-1}(zI - D)^{-1} Q``, and the
    quadrature sum turns ``(z - d)^{-1}`` into ``f(d)``.  ``f`` is evaluated here
    from its geometric-series closed form, not from the nodes."""
    mu = (p.d - p.center) / p.radius
    f = 1.0 / (1.0 + mu ** len(z))
    return np.linalg.solve(p.Q, f[:, None] * (p.Q @ V))


# ---------------------------------------------------------------------------
# Quadrature (eq. 8-4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [4, 16, 32])
@pytest.mark.parametrize("center,radius", [(0.0, 1.0), (1 + 1j, 1.0), (-3 + 0.5j, 2.5)])
def test_trapezoid_filter_is_rational_closed_form(N, center, radius):
    # Half-offset trapezoid nodes z_j = gamma + rho e^{i pi (2j-1)/N} are the
    # roots of (z-gamma)^N = -rho^N, so sum_j w_j/(z_j - lam) = 1/(1 + mu^N),
    # mu = (lam - gamma)/rho (partial fractions of 1/(1+mu^N)).
    z, w = o.contour_nodes(center, radius, N, o.TRAPEZOID)
    rng = np.random.default_rng(1)
    lam = center + radius * (rng.uniform(0, 2.5, 200) * np.exp(2j * np.pi * rng.random(200)))
    mu = (lam - center) / radius
    f = o.filter_function(lam, z, w)
    assert np.max(np.abs(f - 1.0 / (1.0 + mu ** N))) < 1e-12
    # the nodes lie on the circle and the weights sum to the integral of 1/(z - gamma)
    assert np.allclose(np.abs(z - center), radius, atol=1e-14)


def test_gauss_legendre_rule_integrates_the_indicator():
    # The contour integral of 1/(z - lam) is 1 inside and 0 outside the circle;
    # eq. (8-4) with q=16 approximates it well away from the circle.
    z, w = o.contour_nodes(0.5 - 0.2j, 2.0, 16, o.GAUSS_LEGENDRE)
    inside = 0.5 - 0.2j + 2.0 * np.array([0.0, 0.3, 0.2j, -0.25 + 0.1j])
    outside = 0.5 - 0.2j + 2.0 * np.array([3.0, -4.0j, 2.5 + 2.5j])
    assert np.max(np.abs(o.filter_function(inside, z, w) - 1.0)) < 1e-5
    assert np.max(np.abs(o.filter_function(outside, z, w))) < 1e-5
    # nodes: theta_j = (1 + t_j) pi, i.e. the circle traversed once
    assert np.allclose(np.abs(z - (0.5 - 0.2j)), 2.0)
    assert abs(np.sum(w / (z - (0.5 - 0.2j))) - 1.0) < 1e-13


# ---------------------------------------------------------------------------
# The filter against its closed form (Theorem 2.1, eq. 8-3-4)
# ---------------------------------------------------------------------------

def test_filter_matches_weierstrass_closed_form():
    p = pg.workload(1)
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    U = o.apply_filter(o.ShiftedSolver(p.A, p.B, z), w, p.V)
    ref = _closed_form_filter(p, z, w, p.V)
    assert np.linalg.norm(U - ref) / np.linalg.norm(ref) < 1e-11


def test_filter_independent_of_P():
    # Q^{-1} f(D) Q V does not involve P: two pencils sharing Q and D but not P
    # give the same filtered block.
    p = pg.workload(1, n_override=60)
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    rng = np.random.default_rng(3)
    P2 = np.eye(p.n) + 0.1 * (rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))) / math.sqrt(2 * p.n)
    A2 = (P2 * p.d[None, :]) @ p.Q
    B2 = P2 @ p.Q
    U1 = o.apply_filter(o.ShiftedSolver(p.A, p.B, z), w, p.V)
    U2 = o.apply_filter(o.ShiftedSolver(A2, B2, z), w, p.V)
    assert np.linalg.norm(U1 - U2) / np.linalg.norm(U1) < 1e-11


def _explicit_QN(p, z, w):
    return o.apply_filter(o.ShiftedSolver(p.A, p.B, z), w, np.eye(p.n, dtype=np.complex128))


def test_projector_identity_and_geometric_convergence():
    # Eq. (7-26-4): the exact projector satisfies Q^2 = Q.  The N-node filter
    # satisfies Q_N^2 - Q_N = Q^{-1}(f^2 - f)(D) Q, which vanishes geometrically.
    p = pg.make_pencil(16, m=4, inside=3, inside_radius=0.7, outside_r=(1.4, 4.0),
                       c=0.2, seed=11)
    defects = []
    for N in (16, 32, 64, 128):
        z, w = o.contour_nodes(p.center, p.radius, N)
        QN = _explicit_QN(p, z, w)
        f = 1.0 / (1.0 + ((p.d - p.center) / p.radius) ** N)
        ref = np.linalg.solve(p.Q, (f * f - f)[:, None] * p.Q)
        D = QN @ QN - QN
        assert np.linalg.norm(D - ref) <= 1e-11 * max(1.0, np.linalg.norm(ref))
        defects.append(np.linalg.norm(D))
    # each doubling of N at least squares the distance to a projector (|mu| bounded away from 1)
    for a, b in zip(defects, defects[1:]):
        assert b < 0.5 * a or b < 1e-12


def test_trace_of_filter_counts_inside_eigenvalues():
    # Eq. (trace): trace(Q) = s; for Q_N it is sum_i f(d_i).
    p = pg.make_pencil(40, m=4, inside=7, inside_radius=0.8, outside_r=(1.5, 5.0),
                       c=0.1, seed=5)
    z, w = o.contour_nodes(p.center, p.radius, 16)
    QN = _explicit_QN(p, z, w)
    f = 1.0 / (1.0 + ((p.d - p.center) / p.radius) ** 16)
    assert abs(np.trace(QN) - np.sum(f)) < 1e-10
    assert abs(np.trace(QN).real - p.s) < 0.05


# ---------------------------------------------------------------------------
# Projection and reduced pencil (Section 3, Theorem 3.2)
# ---------------------------------------------------------------------------

def test_example31_oblique_projection_finds_printed_eigenpairs():
    A, B, eig = load_example31()
    for t in (2, 3):
        V = pg.start_block(4, t, seed=7 + t)
        res = o.gfeast(A, B, V, 0.0, 1.0, 16, eps=1e-12, max_iter=10)
        assert res.flag == 1
        assert len(res.lam) == 2
        order = np.argsort(res.lam.real)
        for (lam_ref, x_ref), i in zip(sorted(eig, key=lambda e: e[0]), order):
            assert abs(res.lam[i] - lam_ref) < 1e-12
            assert abs(np.vdot(x_ref, res.X[:, i])) > 1 - 1e-12


def test_example31_rayleigh_ritz_collapses():
    # The failure of Example 3.1: with W spanning the filtered subspace, the
    # Rayleigh-Ritz matrices W^* A W and W^* B W vanish (exactly for the exact
    # projector), while the oblique matrices (BW)^* A W do not.
    A, B, _ = load_example31()
    V = pg.start_block(4, 2, seed=3)
    sizes = []
    for N in (16, 32):
        z, w = o.contour_nodes(0.0, 1.0, N)
        W, _ = o.orth(o.apply_filter(o.ShiftedSolver(A, B, z), w, V))
        Ah, Bh = W.conj().T @ A @ W, W.conj().T @ B @ W
        sizes.append(max(np.abs(Ah).max(), np.abs(Bh).max()))
        U2, _ = o.orth(B @ W)
        At, Bt = o.project(A, B, W, U2)
        assert np.abs(Bt).max() > 0.5 and np.abs(At).max() > 0.1
    assert sizes[0] < 1e-3
    assert sizes[1] < 1e-2 * sizes[0]


def test_theorem_3_2_exact_subspace_gives_exact_eigenvalues():
    # With t = s and U spanning the exact eigenspace K = span(Q^{-1}[:, inside]),
    # the reduced pencil's eigenvalues are exactly the inside eigenvalues.
    p = pg.workload(1, n_override=120)
    ins = p.inside_mask
    S = np.linalg.inv(p.Q)
    K = S[:, ins] @ (np.eye(p.s) + 0.3 * pg.start_block(p.s, p.s, seed=2))
    U1, _ = o.orth(K)
    U2, _ = o.orth(p.B @ U1)
    At, Bt = o.project(p.A, p.B, U1, U2)
    a, b, Y = o.reduced_eig(At, Bt)
    lam = np.sort_complex(o.eigenvalues_from(a, b))
    ref = np.sort_complex(p.d[ins])
    assert np.max(np.abs(lam - ref)) < 1e-12
    # and U y are eigenvectors: A x = lam B x
    X = U1 @ Y
    r = o.residuals(p.A, p.B, o.eigenvalues_from(a, b), X)
    assert r.max() < 1e-13


def test_projected_B_equals_R2():
    # U_2^* B U_1 = U_2^* U_2 R_2 = R_2 (QR of B U_1).
    p = pg.workload(1)
    U1, _ = o.orth(p.V)
    U2, R2 = o.orth(p.B @ U1)
    _, Bt = o.project(p.A, p.B, U1, U2)
    assert np.linalg.norm(Bt - R2) / np.linalg.norm(R2) < 1e-14


def test_orth_is_orthonormal_and_reconstructs():
    X = pg.start_block(300, 40, seed=9)
    Qf, R = o.orth(X)
    assert np.linalg.norm(Qf.conj().T @ Qf - np.eye(40)) < 1e-13
    assert np.linalg.norm(Qf @ R - X) / np.linalg.norm(X) < 1e-14
    assert np.all(np.abs(np.tril(R, -1)) == 0)
    assert np.all(np.diag(R).real > 0) and np.all(np.diag(R).imag == 0)


def test_reduced_eig_matches_definition():
    rng = np.random.default_rng(4)
    At = rng.normal(size=(12, 12)) + 1j * rng.normal(size=(12, 12))
    Bt = rng.normal(size=(12, 12)) + 1j * rng.normal(size=(12, 12))
    a, b, Y = o.reduced_eig(At, Bt)
    for i in range(12):
        assert np.linalg.norm(b[i] * At @ Y[:, i] - a[i] * Bt @ Y[:, i]) < 1e-12 * np.linalg.norm(Y[:, i]) * 50
        # eigenvalues are roots of det(At - lam Bt)
        lam = a[i] / b[i]
        sv = np.linalg.svd(At - lam * Bt, compute_uv=False)
        assert sv[-1] / sv[0] < 1e-12


# ---------------------------------------------------------------------------
# The whole algorithm (Algorithm 5)
# ---------------------------------------------------------------------------

def test_n200_two_filters_then_converged_matches_brute_force():
    p = pg.workload(1)
    res2 = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, max_iter=2)
    assert res2.filters == 2 and res2.iters == 2
    assert len(res2.lam) == p.s == 20
    res = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-10, max_iter=20)
    assert res.flag == 1 and res.err < 1e-10 and len(res.lam) == 20
    ev = sla.eigvals(p.A, p.B)
    ref = ev[np.abs(ev - p.center) < p.radius]
    from scipy.optimize import linear_sum_assignment
    C = np.abs(res.lam[:, None] - ref[None, :])
    ri, ci = linear_sum_assignment(C)
    assert np.max(C[ri, ci] / np.maximum(np.abs(ref[ci]), 1e-3)) < 1e-12
    # the generated eigenvalues themselves
    C2 = np.abs(res.lam[:, None] - p.d[p.inside_mask][None, :])
    ri, ci = linear_sum_assignment(C2)
    assert np.max(C2[ri, ci]) < 1e-12
    # eigenvectors are columns of Q^{-1} (Theorem 2.1), up to scale
    S = np.linalg.inv(p.Q)[:, p.inside_mask]
    S = S / np.linalg.norm(S, axis=0)
    for i, j in zip(ri, ci):
        assert abs(np.vdot(S[:, j], res.X[:, i])) > 1 - 1e-10


@pytest.mark.parametrize("k,n", [(2, 800), (5, 512)])
def test_count_and_accuracy_on_scaled_workloads(k, n):
    p = pg.workload(k, n_override=n)
    res = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-10, max_iter=20)
    assert res.flag == 1
    assert len(res.lam) == p.s                                    # P-4: the count
    assert res.err < 1e-10
    assert np.max(o.residuals(p.A, p.B, res.lam, res.X)) < 1e-10
    C = np.abs(res.lam[:, None] - p.d[p.inside_mask][None, :])
    assert np.max(np.min(C, axis=1)) < 1e-10 * max(1.0, abs(p.center))


def test_convergence_rate_prediction():
    # Subspace iteration with the filter: the residual falls per iteration by
    # about |f|_(t+1) / |f|_(s), the ratio of the (t+1)-th and s-th largest |f(d_i)|.
    p = pg.workload(3, n_override=1000)
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    fa = np.sort(np.abs(o.filter_function(p.d, z, w)))[::-1]
    pred = fa[p.m] / fa[p.s - 1]
    res = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-13, max_iter=12)
    es = [h["e"] for h in res.history if h["c"] == p.s and np.isfinite(h["e"]) and h["e"] > 1e-12]
    ratios = [b / a for a, b in zip(es, es[1:])]
    assert len(ratios) >= 2
    obs = float(np.exp(np.mean(np.log(ratios))))
    assert pred / 4 < obs < pred * 4, (pred, obs, ratios)


def test_rebound_returns_previous_iterate():
    # With eps below the attainable floor the run must end on the no-improvement
    # rule (flag 0) or on max_iter, never on convergence; with flag 0 the returned error is the
    # previous iteration's.
    p = pg.workload(1)
    res = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-300, max_iter=30)
    assert res.flag in (0, -1)
    if res.flag == 0:
        assert res.err == res.history[-2]["e"]
        assert res.history[-1]["e"] > res.history[-2]["e"]
    assert len(res.lam) == 20


# ---------------------------------------------------------------------------
# Stopping rules (Algorithm 5, Section 4.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seq,eps,max_iter,flag,stop_k", [
    ([(5, 1e-3), (5, 1e-11)], 1e-10, 10, 1, 2),
    ([(5, 1e-3), (6, 1e-11), (6, 1e-12)], 1e-10, 10, 1, 3),         # count changed at k=2
    ([(5, 1e-3), (5, 1e-6), (5, 1e-5)], 1e-10, 10, 0, 3),           # rebound
    ([(5, 1e-3), (5, 1e-6), (5, 1e-6)], 1e-10, 3, -1, 3),           # equal e: continue
    ([(0, math.inf), (0, math.inf), (4, 1e-4)], 1e-10, 3, -1, 3),   # empty selections
    ([(0, math.inf), (4, 1e-4), (4, 1e-12)], 1e-10, 10, 1, 3),
    ([(3, 1e-3)], 1e-10, 1, -1, 1),
])
def test_stop_rule_sequences(seq, eps, max_iter, flag, stop_k):
    c_prev, e_prev = 0, 0.0
    for k, (c, e) in enumerate(seq, start=1):
        act = o.stop_rule(k, c, e, c_prev, e_prev, eps, max_iter)
        if act != o.CONTINUE:
            assert (act, k) == (flag, stop_k)
            return
        c_prev, e_prev = c, e
    raise AssertionError("sequence did not stop")


# ---------------------------------------------------------------------------
# Eigenvalue derivative (first-order perturbation of a simple eigenvalue)
# ---------------------------------------------------------------------------

def test_gradient_closed_form_and_finite_differences():
    p = pg.workload(5, n_override=64)
    ins = p.inside_mask
    # Closed form for A = P D Q, B = P Q: x_i = Q^{-1} e_i, y_i = P^{-*} e_i, y_i^* B x_i = 1
    Qi, Pi = np.linalg.inv(p.Q), np.linalg.inv(p.P)
    lam_in = np.where(ins, p.d, 0)
    GA_ref = 2.0 * Pi.conj().T @ np.diag(lam_in) @ Qi.conj().T
    GB_ref = -2.0 * Pi.conj().T @ np.diag(np.abs(lam_in) ** 2) @ Qi.conj().T
    # oracle's gradient from brute-force left/right eigenvectors
    ev, Yl, X = sla.eig(p.A, p.B, left=True, right=True)
    sel = np.abs(ev - p.center) < p.radius
    GA, GB = o.loss_gradient(p.B, ev[sel], X[:, sel], Yl[:, sel])
    assert np.linalg.norm(GA - GA_ref) / np.linalg.norm(GA_ref) < 1e-10
    assert np.linalg.norm(GB - GB_ref) / np.linalg.norm(GB_ref) < 1e-10

    def loss(A, B):
        e = sla.eigvals(A, B)
        e = e[np.abs(e - p.center) < p.radius]
        return float(np.sum(np.abs(e) ** 2))

    rng = np.random.default_rng(8)
    h = 1e-6
    for _ in range(4):
        dA = rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))
        dB = rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))
        nr = math.sqrt(np.linalg.norm(dA) ** 2 + np.linalg.norm(dB) ** 2)
        dA, dB = dA / nr, dB / nr
        fd = (loss(p.A + h * dA, p.B + h * dB) - loss(p.A - h * dA, p.B - h * dB)) / (2 * h)
        an = np.real(np.vdot(GA, dA)) + np.real(np.vdot(GB, dB))
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an))


def _closed_form_left(p, X):
    """Left eigenvectors of ``A = P D Q``, ``B = P Q`` matching the columns of
    ``X``: ``x = Q^{-1} e_k alpha`` gives ``y = P^{-*} e_k / conj(alpha)`` with
    ``y^* B x = 1``; ``k`` is the index whose coordinate dominates ``Q x``."""
    QX = p.Q @ X
    Pi_h = np.linalg.inv(p.P).conj().T
    Y = np.zeros_like(X)
    for i in range(X.shape[1]):
        k = int(np.argmax(np.abs(QX[:, i])))
        Y[:, i] = Pi_h[:, k] / np.conj(QX[k, i])
    return Y


@pytest.mark.parametrize("n", [64, 300])
def test_left_eigenvectors_match_closed_form(n):
    # The adjoint filter operator sum_j conj(w_j)(z_j B - A)^{-*} B^* scales each
    # left eigenvector P^{-*} e_k by conj(f(d_k)); three sweeps from the converged
    # right eigenvectors reach the closed form to rounding.
    p = pg.workload(5, n_override=n)
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    res = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-13, max_iter=20)
    assert len(res.lam) == p.s
    Y = o.left_eigenvectors(o.ShiftedSolver(p.A, p.B, z), w, p.B, res.X, 3)
    Yc = _closed_form_left(p, res.X)
    assert np.linalg.norm(Y - Yc) / np.linalg.norm(Yc) < 1e-12
    assert np.abs(Y.conj().T @ p.B @ res.X - np.eye(p.s)).max() < 1e-12


# ---------------------------------------------------------------------------
# Residual of eq. (5-1), worked by hand on Example 3.1
# ---------------------------------------------------------------------------

def _residual_planted_denominator(A, B, lam, X):
    """A plausible mistake in eq. (5-1): the denominator ||A x|| + |lambda| ||B x||."""
    AX, BX = A @ X, B @ X
    return np.array([np.linalg.norm(AX[:, i] - lam[i] * BX[:, i]) /
                     (np.linalg.norm(AX[:, i]) + abs(lam[i]) * np.linalg.norm(BX[:, i]))
                     for i in range(X.shape[1])])


# (x, lambda, r) with r worked out by hand for the pencil of Example 3.1:
#  x = e1 + 0.1 e2, lambda = 0.2:  A x = (0, 0, 0.05, 0.2), B x = (0, 0, 0.1, 1),
#    A x - lambda B x = (0, 0, 0.03, 0)  ->  r = 0.03 / (sqrt(0.0425) + sqrt(1.01));
#  x = e1 + i e2, lambda = 0.2 + 0.1i:  A x = (0, 0, 0.5i, 0.2), B x = (0, 0, i, 1),
#    A x - lambda B x = (0, 0, 0.1 + 0.3i, -0.1i)  ->  r = sqrt(0.11) / (sqrt(0.29) + sqrt(2)).
_EX31_RESIDUALS = [
    (np.array([1, 0.1, 0, 0], dtype=np.complex128), 0.2,
     0.03 / (math.sqrt(0.0425) + math.sqrt(1.01))),
    (np.array([1, 1j, 0, 0], dtype=np.complex128), 0.2 + 0.1j,
     math.sqrt(0.11) / (math.sqrt(0.29) + math.sqrt(2.0))),
]


def test_residual_eq_5_1_hand_values_on_example31():
    # Eq. (5-1): r = ||A x - lambda B x||_2 / (||A x||_2 + ||B x||_2), checked on
    # values worked out by hand (no re-typed formula), scale invariance in x,
    # zero at the printed eigenpairs and +inf for an infinite eigenvalue.
    A, B, eig = load_example31()
    X = np.stack([x for x, _, _ in _EX31_RESIDUALS], axis=1)
    lam = np.array([l for _, l, _ in _EX31_RESIDUALS])
    ref = np.array([r for _, _, r in _EX31_RESIDUALS])
    r = o.residuals(A, B, lam, X)
    assert np.max(np.abs(r - ref) / ref) < 1e-14
    assert np.max(np.abs(o.residuals(A, B, lam, (2.5 - 1.5j) * X) - ref) / ref) < 1e-14
    for l, x in eig:
        assert o.residuals(A, B, np.array([l]), x[:, None])[0] == 0.0
    assert o.residuals(A, B, np.array([np.inf + 0j]), X[:, :1])[0] == np.inf


def test_planted_residual_denominator_is_caught():
    # The hand values above reject the denominator ||A x|| + |lambda| ||B x||.
    A, B, _ = load_example31()
    X = np.stack([x for x, _, _ in _EX31_RESIDUALS], axis=1)
    lam = np.array([l for _, l, _ in _EX31_RESIDUALS])
    ref = np.array([r for _, _, r in _EX31_RESIDUALS])
    bad = _residual_planted_denominator(A, B, lam, X)
    assert np.min(np.abs(bad - ref) / ref) > 0.1


# ---------------------------------------------------------------------------
# Eigenvalue derivatives (first-order perturbation of a simple eigenvalue)
# ---------------------------------------------------------------------------

def _brute_force_pairs(A, B, center, radius, seed):
    """Inside eigenvalues with right and left eigenvectors from the dense QZ,
    each vector rescaled by a random complex factor (so y^* B x != 1)."""
    ev, Yl, X = sla.eig(A, B, left=True, right=True)
    sel = np.abs(ev - center) < radius
    rng = np.random.default_rng(seed)
    k = int(np.count_nonzero(sel))
    sx = rng.uniform(0.5, 2.0, k) * np.exp(2j * np.pi * rng.random(k))
    sy = rng.uniform(0.5, 2.0, k) * np.exp(2j * np.pi * rng.random(k))
    return ev[sel], X[:, sel] * sx[None, :], Yl[:, sel] * sy[None, :]


def _fd_eigenvalue_derivative(A, B, lam, dA, dB, h, center, radius):
    """Central differences of the brute-force eigenvalues along (dA, dB), each
    perturbed eigenvalue matched to the nearest unperturbed one."""
    out = []
    for sgn in (1.0, -1.0):
        e = sla.eigvals(A + sgn * h * dA, B + sgn * h * dB)
        e = e[np.isfinite(e)]
        out.append(np.array([e[np.argmin(np.abs(e - l))] for l in lam]))
    return (out[0] - out[1]) / (2.0 * h)


def test_eigenvalue_derivatives_match_finite_differences():
    # d lambda_i = y_i^*(dA - lambda_i dB) x_i / (y_i^* B x_i) against central
    # differences of brute-force eigenvalues of the perturbed pencils, with the
    # eigenvectors scaled arbitrarily (the quotient must not depend on it).
    p = pg.workload(5, n_override=48)
    lam, X, Yl = _brute_force_pairs(p.A, p.B, p.center, p.radius, seed=12)
    assert lam.size == p.s
    rng = np.random.default_rng(13)
    for _ in range(3):
        dA = rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))
        dB = rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))
        an = o.eigenvalue_derivatives(p.B, lam, X, Yl, dA, dB)
        fd = _fd_eigenvalue_derivative(p.A, p.B, lam, dA, dB, 1e-6, p.center, p.radius)
        assert np.max(np.abs(an - fd) / np.abs(fd)) < 1e-6


def test_eigenvalue_derivatives_closed_form_PDQ():
    # For A = P D Q, B = P Q: x_i = Q^{-1} e_i, y_i = P^{-*} e_i, so
    # d lambda_i = e_i^T P^{-1} (dA - d_i dB) Q^{-1} e_i, the i-th diagonal entry
    # of the transformed perturbation (Theorem 2.1's Weierstrass form).
    p = pg.workload(5, n_override=64)
    ins = np.flatnonzero(p.inside_mask)
    Pi, Qi = np.linalg.inv(p.P), np.linalg.inv(p.Q)
    rng = np.random.default_rng(14)
    dA = rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))
    dB = rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))
    TA, TB = Pi @ dA @ Qi, Pi @ dB @ Qi
    ref = np.diag(TA)[ins] - p.d[ins] * np.diag(TB)[ins]
    # oracle from brute-force (arbitrarily scaled) eigenvectors
    lam, X, Yl = _brute_force_pairs(p.A, p.B, p.center, p.radius, seed=15)
    order = [int(np.argmin(np.abs(lam - p.d[i]))) for i in ins]
    an = o.eigenvalue_derivatives(p.B, lam[order], X[:, order], Yl[:, order], dA, dB)
    assert np.max(np.abs(an - ref) / np.abs(ref)) < 1e-10


def test_planted_eigenvalue_derivative_mistakes_are_caught():
    # Dropping the denominator y^* B x, flipping the sign of the dB term or
    # conjugating lambda in it all fail the finite-difference pin.
    p = pg.workload(5, n_override=48)
    lam, X, Yl = _brute_force_pairs(p.A, p.B, p.center, p.radius, seed=16)
    rng = np.random.default_rng(17)
    dA = rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))
    dB = rng.normal(size=(p.n, p.n)) + 1j * rng.normal(size=(p.n, p.n))
    fd = _fd_eigenvalue_derivative(p.A, p.B, lam, dA, dB, 1e-6, p.center, p.radius)
    planted = [
        lambda x, y, l: np.vdot(y, (dA - l * dB) @ x),                          # no denominator
        lambda x, y, l: np.vdot(y, (dA + l * dB) @ x) / np.vdot(y, p.B @ x),    # sign of dB
        lambda x, y, l: np.vdot(y, (dA - np.conj(l) * dB) @ x) / np.vdot(y, p.B @ x),
    ]
    for f in planted:
        bad = np.array([f(X[:, i], Yl[:, i], lam[i]) for i in range(lam.size)])
        assert np.max(np.abs(bad - fd) / np.abs(fd)) > 1e-3


# ---------------------------------------------------------------------------
# Planted mistakes: the pins above must catch them
# ---------------------------------------------------------------------------

def test_planted_adjoint_without_B_star_stalls():
    # Sweeping the adjoint resolvent sum without B^* between the sweeps stalls at
    # about max|f| outside times the departure of B from I; the closed-form pin
    # rejects it.
    p = pg.workload(5, n_override=300)
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    res = o.gfeast(p.A, p.B, p.V, p.center, p.radius, p.nodes, eps=1e-13, max_iter=20)
    S = o.ShiftedSolver(p.A, p.B, z)
    W = p.B @ res.X
    for _ in range(4):
        W = o.apply_filter_adjoint(S, w, W)
    Y = W @ np.linalg.inv(W.conj().T @ p.B @ res.X).conj().T
    Yc = _closed_form_left(p, res.X)
    assert np.linalg.norm(Y - Yc) / np.linalg.norm(Yc) > 1e-10


def test_planted_weight_sign_error_is_caught():
    p = pg.workload(1, n_override=80)
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    ref = _closed_form_filter(p, z, w, p.V)
    bad = o.apply_filter(o.ShiftedSolver(p.A, p.B, z), -w, p.V)        # sign flipped
    assert np.linalg.norm(bad - ref) / np.linalg.norm(ref) > 0.5
    z2 = p.center + p.radius * np.exp(2j * np.pi * np.arange(p.nodes) / p.nodes)   # unshifted nodes
    bad2 = o.apply_filter(o.ShiftedSolver(p.A, p.B, z2), (z2 - p.center) / p.nodes, p.V)
    assert np.linalg.norm(bad2 - ref) / np.linalg.norm(ref) > 1e-3


def test_planted_rayleigh_ritz_fails_example31():
    # Using the trial space as test space (Rayleigh-Ritz) instead of B K breaks
    # the method on Example 3.1: the reduced pencil is numerically zero.
    A, B, _ = load_example31()
    z, w = o.contour_nodes(0.0, 1.0, 32)
    U1, _ = o.orth(o.apply_filter(o.ShiftedSolver(A, B, z), w, pg.start_block(4, 2, seed=1)))
    At, Bt = o.project(A, B, U1, U1)
    assert np.abs(At).max() < 1e-8 and np.abs(Bt).max() < 1e-8


# ---------------------------------------------------------------------------
# Generator sanity (inputs shared by both sides)
# ---------------------------------------------------------------------------

def test_generator_regions_and_counts():
    p = pg.workload(2, n_override=400)
    assert p.s == 10
    out = np.abs(p.d[~p.inside_mask] - p.center)
    assert out.min() >= 1.3 and out.max() < 10.0
    q = pg.workload(3, n_override=400)
    r = np.abs(q.d - q.center)
    assert np.count_nonzero(r < 1.0) == q.s
    assert np.count_nonzero((r >= 1.05) & (r < 1.2)) == round(0.05 * (400 - q.s))
    # deterministic
    p2 = pg.workload(2, n_override=400)
    assert np.array_equal(p.A, p2.A) and np.array_equal(p.V, p2.V)
    # Weierstrass structure: B^{-1} A = Q^{-1} D Q
    assert np.linalg.norm(np.linalg.solve(p.B, p.A) @ np.linalg.inv(p.Q) - np.linalg.inv(p.Q) * p.d[None, :]) < 1e-10
