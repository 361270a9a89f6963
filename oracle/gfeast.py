"""Plain FP64 CPU oracle of the oblique-projection FEAST method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the package
``paper_1404_1768_amd``) may import, call or link this module; only the tests,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the GPU path: its only dependencies are NumPy and SciPy
(LAPACK ``zgetrf``/``zgetrs`` for the shifted solves, Householder QR, ``zggev``
for the reduced pencil), as the paper's own MATLAB experiments use ``lu`` plus
triangular substitution and an ``xGGEV``-type solver.

Everything is complex128, row-major (NumPy's default order), and follows the
paper step by step; citations name the section, equation or algorithm.

Readings of the paper taken here (each is listed with its reason in the design
notes of the repository):

* Quadrature: the trapezoid rule with half-offset nodes
  ``theta_j = 2 pi (j - 1/2) / N``, ``w_j = (z_j - gamma)/N`` discretises the
  circle integral of eq. (8-4); Gauss-Legendre with ``theta_j = (1 + t_j) pi``
  and ``w_j = omega_j (z_j - gamma)/2`` is eq. (8-4) itself.
* Sign: shifted systems are ``(z_j B - A) Y_j = B U_1`` as in eq. (4-4).
* GFEAST's Search call with a fixed subspace size ``t = m`` and a caller-supplied
  start block ``V``: ``U_1`` is the orthonormal factor of the filtered block
  ``Q_N V`` (the remark after Algorithm 4: its ``U_1`` is a projection onto the
  eigenspace, i.e. the first filter application).  ``search`` is Algorithm 4
  itself; its random columns come from a caller-supplied pool, its trace
  estimate uses the real part of ``trace(Y_0^* U)`` (the expectation is real),
  and the numerical rank of the column-pivoted ``R`` counts the diagonal
  entries with ``|R_ii| >= tau |R_11|`` (the paper names rank-revealing QR but
  no threshold).
* The QR step at the end of each iteration factors ``B U_1`` with the new
  ``U_1`` (same span as ``B U``).
* Empty selection: ``e(k) = +inf`` and the two rules that compare ``c(k)``
  with ``c(k-1)`` are skipped.
* ``lambda`` inside means ``|lambda - gamma| < rho`` (strict); infinite
  eigenvalues (``beta = 0``) are outside.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg as sla

TRAPEZOID = 0
GAUSS_LEGENDRE = 1


# ---------------------------------------------------------------------------
# Quadrature on the circle (eq. 8-4, Section 4.3)
# ---------------------------------------------------------------------------

def contour_nodes(center: complex, radius: float, N: int, rule: int = TRAPEZOID):
    """Nodes ``z_j`` and weights ``w_j`` so that
    ``(1/(2 pi i)) \\oint g(z) dz  ~=  sum_j w_j g(z_j)`` on the circle.

    With ``z = gamma + rho e^{i theta}`` one has ``dz/(2 pi i) = (z-gamma) dtheta/(2 pi)``.
    Trapezoid: ``theta_j = 2 pi (j - 1/2)/N``, ``w_j = (z_j - gamma)/N``.
    Gauss-Legendre (eq. 8-4): ``theta_j = (1 + t_j) pi``, ``w_j = omega_j (z_j - gamma)/2``.
    """
    if N < 1:
        raise ValueError("N must be positive")
    center = complex(center)
    if rule == TRAPEZOID:
        theta = 2.0 * math.pi * (np.arange(1, N + 1) - 0.5) / N
        z = center + radius * np.exp(1j * theta)
        w = (z - center) / N
    elif rule == GAUSS_LEGENDRE:
        t, om = np.polynomial.legendre.leggauss(N)
        theta = (1.0 + t) * math.pi
        z = center + radius * np.exp(1j * theta)
        w = 0.5 * om * (z - center)
    else:
        raise ValueError("unknown quadrature rule")
    return z.astype(np.complex128), w.astype(np.complex128)


def filter_function(lam, z, w):
    """Scalar filter of the discretised projector: ``f(lam) = sum_j w_j / (z_j - lam)``.

    Applying the quadrature of eq. (8-4) to the resolvent of eq. (8-3-4) maps an
    eigenvalue ``lam`` of the pencil to ``f(lam)``.
    """
    lam = np.asarray(lam, dtype=np.complex128)
    return np.sum(w[:, None] / (z[:, None] - lam.reshape(1, -1)), axis=0).reshape(lam.shape)


# ---------------------------------------------------------------------------
# The filter: shifted solves and weighted sum (eqs. 8-4, 4-4; LU reuse, Section 4.3)
# ---------------------------------------------------------------------------

class ShiftedSolver:
    """LU factors of ``z_j B - A`` for every node, computed once and reused by
    every later filter application (Section 4.3: the factors of eq. (4-4) are
    reused in subsequent iterations)."""

    def __init__(self, A: np.ndarray, B: np.ndarray, z: np.ndarray):
        self.A, self.B, self.z = A, B, z
        self._lu: List = [None] * len(z)

    def factor(self, j: int):
        if self._lu[j] is None:
            M = self.z[j] * self.B - self.A                     # eq. (4-4)
            self._lu[j] = sla.lu_factor(M, check_finite=False)  # LAPACK zgetrf
        return self._lu[j]

    def solve(self, j: int, R: np.ndarray, trans: int = 0) -> np.ndarray:
        """``(z_j B - A)^{-1} R`` (``trans=2``: ``(z_j B - A)^{-H} R``)."""
        return sla.lu_solve(self.factor(j), R, trans=trans, check_finite=False)


def apply_filter(solver: ShiftedSolver, w: np.ndarray, U1: np.ndarray,
                 BU1: Optional[np.ndarray] = None) -> np.ndarray:
    """``U = sum_j w_j (z_j B - A)^{-1} B U_1`` (eq. 8-4 with the systems of eq. 4-4)."""
    R = solver.B @ U1 if BU1 is None else BU1
    U = np.zeros_like(R)
    for j in range(len(w)):
        U += w[j] * solver.solve(j, R)
    return U


def apply_filter_adjoint(solver: ShiftedSolver, w: np.ndarray, W: np.ndarray) -> np.ndarray:
    """``sum_j conj(w_j) (z_j B - A)^{-H} W`` -- the conjugate transpose of the
    resolvent sum of eq. (8-4) without its trailing ``B``.  For a left
    eigenvector ``y_k`` (``y_k^H A = lam_k y_k^H B``) one has
    ``(z_j B - A)^H y_k = conj(z_j - lam_k) B^H y_k``, so this maps ``B^H y_k``
    to ``conj(f(lam_k)) y_k``."""
    out = np.zeros_like(W)
    for j in range(len(w)):
        out += np.conj(w[j]) * solver.solve(j, W, trans=2)
    return out


def left_eigenvectors(solver: ShiftedSolver, w: np.ndarray, B: np.ndarray, X: np.ndarray,
                      sweeps: int) -> np.ndarray:
    """Left eigenvectors belonging to the right eigenvectors ``X`` found inside
    the contour: subspace iteration with the adjoint filter operator
    ``W -> sum_j conj(w_j) (z_j B - A)^{-H} B^H W`` from ``W = X`` (it scales
    each left eigenvector ``y_k`` by ``conj(f(lam_k))``, so the components
    outside the contour shrink by the filter values there), then the
    normalisation ``Y = W (W^H B X)^{-H}`` that makes ``Y^H B X = I``."""
    W = X
    for _ in range(sweeps):
        W = apply_filter_adjoint(solver, w, B.conj().T @ W)
    return W @ np.linalg.inv(W.conj().T @ B @ X).conj().T


# ---------------------------------------------------------------------------
# Orthonormalisation, projection and the reduced pencil (Algorithms 3 and 5)
# ---------------------------------------------------------------------------

def orth(X: np.ndarray):
    """Householder QR ``X = Q R`` with the diagonal of ``R`` made real and
    non-negative, so that ``Q`` and ``R`` are unique when ``X`` has full rank."""
    Qf, R = np.linalg.qr(X, mode="reduced")
    dg = np.diag(R)
    ph = np.where(np.abs(dg) > 0, dg / np.where(np.abs(dg) > 0, np.abs(dg), 1.0), 1.0)
    Qf = Qf * ph[None, :]
    R = np.conj(ph)[:, None] * R
    return Qf, R


def project(A: np.ndarray, B: np.ndarray, U1: np.ndarray, U2: np.ndarray):
    """Oblique projection with trial space span(U_1) and test space span(U_2) = B K
    (eqs. 6-3-12, 6-3-13, 7-10; the reduced pencil of Algorithm 5):
    ``At = U_2^* A U_1``, ``Bt = U_2^* B U_1``."""
    U2h = U2.conj().T
    return U2h @ (A @ U1), U2h @ (B @ U1)


def reduced_eig(At: np.ndarray, Bt: np.ndarray):
    """All eigenpairs of the t x t pencil ``At y = lambda Bt y`` (LAPACK zggev,
    Section 3).  Returns homogeneous ``(alpha, beta)`` and right eigenvectors."""
    ab, Y = sla.eig(At, Bt, right=True, homogeneous_eigvals=True, check_finite=False)
    return ab[0], ab[1], Y


def eigenvalues_from(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = np.where(beta != 0, alpha / np.where(beta != 0, beta, 1.0), np.inf + 0j)
    return lam


def normalize_columns(X: np.ndarray) -> np.ndarray:
    """Unit 2-norm columns whose largest-modulus entry is real and positive."""
    X = X.copy()
    for i in range(X.shape[1]):
        nr = np.linalg.norm(X[:, i])
        if nr == 0:
            continue
        k = int(np.argmax(np.abs(X[:, i])))
        X[:, i] *= np.conj(X[k, i]) / (abs(X[k, i]) * nr)
    return X


def residuals(A: np.ndarray, B: np.ndarray, lam: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Relative residuals ``r_i = ||A x_i - lambda_i B x_i|| / (||A x_i|| + ||B x_i||)``
    (eq. 5-1; Algorithm 5's residual).  Infinite ``lambda_i`` give ``+inf``."""
    AX, BX = A @ X, B @ X
    r = np.full(X.shape[1], np.inf)
    for i in range(X.shape[1]):
        if not np.isfinite(lam[i]):
            continue
        num = np.linalg.norm(AX[:, i] - lam[i] * BX[:, i])
        den = np.linalg.norm(AX[:, i]) + np.linalg.norm(BX[:, i])
        r[i] = num / den if den > 0 else np.inf
    return r


def inside(lam: np.ndarray, center: complex, radius: float) -> np.ndarray:
    """Strictly inside the circle; infinite values are outside."""
    lam = np.asarray(lam)
    ok = np.isfinite(lam)
    out = np.zeros(lam.shape, dtype=bool)
    out[ok] = np.abs(lam[ok] - center) < radius
    return out


# ---------------------------------------------------------------------------
# Stopping rules (Algorithm 5; Section 4.2)
# ---------------------------------------------------------------------------

CONTINUE = 2
CONVERGED = 1      # same count and e(k) < eps
REBOUND = 0        # same count and e(k) > e(k-1): previous iterate is returned
MAX_ITER = -1      # k = max_iter


def stop_rule(k: int, c_k: int, e_k: float, c_prev: int, e_prev: float,
              eps: float, max_iter: int) -> int:
    """Decision after iteration ``k``.  Rules 13 and 14 need ``c(k) = c(k-1)``;
    they are skipped when nothing was selected (``c(k) = 0``), since
    ``e(k) = max([])`` is undefined.  Rule 13 is tested before 14 and 14 uses a
    strict increase."""
    if c_k > 0 and c_k == c_prev:
        if e_k < eps:
            return CONVERGED
        if e_k > e_prev:
            return REBOUND
    if k == max_iter:
        return MAX_ITER
    return CONTINUE


# ---------------------------------------------------------------------------
# GFEAST (Algorithm 5) with a fixed subspace size
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    lam: np.ndarray                 # selected eigenvalues Lambda
    X: np.ndarray                   # selected eigenvectors (unit columns)
    r: np.ndarray                   # their residuals
    err: float                      # Err
    flag: int                       # 1 / 0 / -1
    iters: int                      # k at which it stopped
    filters: int                    # filter applications performed
    history: List[Dict] = dataclasses.field(default_factory=list)


def gfeast(A: np.ndarray, B: np.ndarray, V: np.ndarray, center: complex, radius: float,
           N: int, rule: int = TRAPEZOID, eps: float = 1e-10, eta: float = 1e-3,
           max_iter: int = 20, solver: Optional[ShiftedSolver] = None) -> Result:
    """Algorithm 5 with ``t = V.shape[1]`` fixed.

    The Search call becomes one filter application of the start block ``V``
    followed by QR; the rest follows Algorithm 5 in order.
    """
    z, w = contour_nodes(center, radius, N, rule)
    if solver is None:
        solver = ShiftedSolver(A, B, z)
    # Search with fixed t: U = Q_N V, U_1 = orth(U)
    U = apply_filter(solver, w, V)
    U1, _ = orth(U)
    return gfeast_from(A, B, U1, center, radius, N, rule, eps, eta, max_iter, solver, filters=1)


def gfeast_from(A: np.ndarray, B: np.ndarray, U1: np.ndarray, center: complex, radius: float,
                N: int, rule: int = TRAPEZOID, eps: float = 1e-10, eta: float = 1e-3,
                max_iter: int = 20, solver: Optional[ShiftedSolver] = None,
                filters: int = 0) -> Result:
    """Algorithm 5 after its Search call, from an orthonormal ``U_1`` that is
    already a filtered basis (Search's output, or that of ``gfeast``)."""
    z, w = contour_nodes(center, radius, N, rule)
    if solver is None:
        solver = ShiftedSolver(A, B, z)
    # QR of B U_1 = U_2 R_2
    BU1 = B @ U1
    U2, _ = orth(BU1)
    # e(0) = 0, c(0) = 0
    e_prev, c_prev = 0.0, 0
    prev = None
    history = []
    for k in range(1, max_iter + 1):
        # reduced pencil
        At = U2.conj().T @ (A @ U1)
        Bt = U2.conj().T @ BU1
        # reduced eigenproblem and Ritz vectors
        alpha, beta, Y = reduced_eig(At, Bt)
        lam = eigenvalues_from(alpha, beta)
        X = normalize_columns(U1 @ Y)
        # residuals and selection, c(k)
        r = residuals(A, B, lam, X)
        sel = inside(lam, center, radius) & (r < eta)
        c_k = int(np.count_nonzero(sel))
        # e(k) = max r
        e_k = float(np.max(r[sel])) if c_k > 0 else math.inf
        cur = (lam[sel], X[:, sel], r[sel], e_k)
        history.append({"k": k, "c": c_k, "e": e_k})
        # stopping rules
        act = stop_rule(k, c_k, e_k, c_prev, e_prev, eps, max_iter)
        if act == CONVERGED or act == MAX_ITER:
            return Result(cur[0], cur[1], cur[2], cur[3], act, k, filters, history)
        if act == REBOUND:
            return Result(prev[0], prev[1], prev[2], prev[3], act, k, filters, history)
        prev = cur
        e_prev, c_prev = e_k, c_k
        # filter: U = Q_N U_1 with the cached factors
        U = apply_filter(solver, w, U1, BU1)
        filters += 1
        # QR of U and of B U
        U1, _ = orth(U)
        BU1 = B @ U1
        U2, _ = orth(BU1)
    raise AssertionError("unreachable: the iteration cap stops at max_iter")


# ---------------------------------------------------------------------------
# Block_CIRR (Algorithm 1, Section 2): the comparison method on the same solves
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class CirrResult:
    lam: np.ndarray     # selected eigenvalues (inside the circle, r < eta)
    X: np.ndarray       # their eigenvectors (unit columns)
    r: np.ndarray       # their residuals (eq. 5-1)
    t: int              # columns of the moment block, h g
    sv: np.ndarray      # singular values of the moment block


def cirr_moments(solver: ShiftedSolver, z: np.ndarray, w: np.ndarray, Y: np.ndarray,
                 g: int, center: complex, radius: float) -> np.ndarray:
    """Moments of Algorithm 1: ``[R_0, ..., R_{g-1}]`` with ``R_i`` the quadrature of
    ``F_i Y`` (eq. 2-2-21), in the shifted and scaled powers
    ``((z - gamma)/rho)^i`` (same span as ``z^i`` for ``i < g``)."""
    mu = (z - center) / radius
    Ys = [solver.solve(j, Y) for j in range(len(w))]
    return np.hstack([sum(w[j] * mu[j] ** i * Ys[j] for j in range(len(w))) for i in range(g)])


def block_cirr(A: np.ndarray, B: np.ndarray, Y: np.ndarray, g: int, center: complex,
               radius: float, N: int, rule: int = TRAPEZOID, eta: float = 1e-3,
               solver: Optional[ShiftedSolver] = None) -> CirrResult:
    """Algorithm 1: moments, SVD (all ``h g`` left singular vectors),
    Rayleigh-Ritz with the left space equal to the right one, Ritz vectors and
    the final selection (inside the circle with ``r_i < eta``, as in GFEAST's
    selection)."""
    z, w = contour_nodes(center, radius, N, rule)
    if solver is None:
        solver = ShiftedSolver(A, B, z)
    M = cirr_moments(solver, z, w, Y, g, center, radius)
    U, S, _ = np.linalg.svd(M, full_matrices=False)
    Ab = U.conj().T @ (A @ U)
    Bb = U.conj().T @ (B @ U)
    alpha, beta, Yv = reduced_eig(Ab, Bb)
    lam = eigenvalues_from(alpha, beta)
    X = normalize_columns(U @ Yv)
    r = residuals(A, B, lam, X)
    sel = inside(lam, center, radius) & (r < eta)
    return CirrResult(lam[sel], X[:, sel], r[sel], M.shape[1], S)


# ---------------------------------------------------------------------------
# Reference spectrum and contours for the sparse-shaped stand-ins (Table 1)
# ---------------------------------------------------------------------------

def dense_eigenvalues(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """All finite eigenvalues of the pencil by the dense QZ (LAPACK ``xGGEV``),
    the reference the paper's experiments take (Section 5).  A pencil with real
    entries is passed to the real QZ (``dggev``), whose eigenvalues are the same
    and which runs several times faster."""
    if not np.iscomplexobj(A) or (np.all(A.imag == 0) and np.all(B.imag == 0)):
        A, B = np.real(A), np.real(B)
    lam = sla.eigvals(A, B)
    return lam[np.isfinite(lam)]


def standin_contour(lam: np.ndarray, target: int = 20, probes: int = 40):
    """A circle around about ``target`` reference eigenvalues with the widest
    relative gap: centres at the ``probes`` eigenvalues closest to the median
    real part, counts ``target - 8 .. target + 8``, radius midway between the
    s-th and (s+1)-th distances.  Returns (center, radius, s, gap)."""
    best = None
    for c in lam[np.argsort(np.abs(lam - np.median(lam.real)))[:probes]]:
        d = np.sort(np.abs(lam - c))
        for s in range(max(8, target - 8), min(target + 9, d.size)):
            gap = d[s] / d[s - 1]
            if best is None or gap > best[3]:
                best = (complex(c), float(0.5 * (d[s - 1] + d[s])), s, float(gap))
    return best


# ---------------------------------------------------------------------------
# Irregular contours (Section 4.3): an enclosing circle, then the region test
# ---------------------------------------------------------------------------

def enclosing_circle(vertices: np.ndarray, margin: float = 0.0):
    """Smallest circle containing all vertices, by brute force over the circles
    spanned by two points (as a diameter) or three (circumcircle); the radius
    is then enlarged by ``1 + margin``.  (A disc containing the vertices
    contains the polygon: it is convex.)  Small polygons only."""
    v = np.asarray(vertices, dtype=np.complex128).ravel()
    if v.size == 1:
        return complex(v[0]), 0.0
    cands = []
    for i in range(v.size):
        for j in range(i + 1, v.size):
            cands.append(((v[i] + v[j]) / 2, abs(v[i] - v[j]) / 2))
            for k in range(j + 1, v.size):
                a, b, c = v[i], v[j], v[k]
                # circumcentre: the point equidistant from a, b, c (2x2 linear system)
                M = np.array([[2 * (b - a).real, 2 * (b - a).imag],
                              [2 * (c - a).real, 2 * (c - a).imag]])
                if abs(np.linalg.det(M)) < 1e-300:
                    continue
                rhs = np.array([abs(b) ** 2 - abs(a) ** 2, abs(c) ** 2 - abs(a) ** 2])
                x, y = np.linalg.solve(M, rhs)
                cands.append((complex(x, y), abs(complex(x, y) - a)))
    best = None
    for c, r in cands:
        if np.all(np.abs(v - c) <= r * (1 + 1e-10) + 1e-14) and (best is None or r < best[1]):
            best = (c, r)
    return complex(best[0]), float(best[1]) * (1.0 + margin)


def inside_region(points: np.ndarray, vertices: np.ndarray) -> np.ndarray:
    """Winding number of the closed polygon about each point (non-zero =
    inside), summed from the turning angles of its edges."""
    v = np.asarray(vertices, dtype=np.complex128).ravel()
    z = np.asarray(points, dtype=np.complex128).ravel()
    a = v[None, :] - z[:, None]
    b = np.roll(v, -1)[None, :] - z[:, None]
    wind = np.sum(np.angle(b / a), axis=1) / (2 * np.pi)
    return np.abs(wind) > 0.5


def gfeast_region(A: np.ndarray, B: np.ndarray, V: np.ndarray, vertices: np.ndarray, N: int,
                  margin: float = 0.1, **kw):
    """Section 4.3 for an irregular curve: Algorithm 5 on an enclosing circle,
    then the eigenpairs inside the curve.  Returns (Result restricted, circle)."""
    center, radius = enclosing_circle(vertices, margin)
    res = gfeast(A, B, V, center, radius, N, **kw)
    keep = inside_region(res.lam, vertices)
    return dataclasses.replace(res, lam=res.lam[keep], X=res.X[:, keep], r=res.r[keep]), \
        (center, radius)


# ---------------------------------------------------------------------------
# Search (Algorithm 4, Section 4.1): an upper bound t of s and U_1
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SearchResult:
    U1: np.ndarray      # orthonormal basis of the filtered block (n x t)
    t: int              # numerical rank at the last round (upper bound of s)
    s0: int             # trace estimate of s
    rounds: int         # rank-revealing tests performed
    used: int           # pool columns consumed
    filters: int        # filter applications


def numerical_rank(R: np.ndarray, tau: float) -> int:
    """Number of diagonal entries of a column-pivoted triangular factor with
    ``|R_ii| >= tau |R_11|`` (pivoting makes them non-increasing)."""
    d = np.abs(np.diag(R))
    if d.size == 0 or not d[0] > 0:
        return 0
    return int(np.count_nonzero(d >= tau * d[0]))


def trace_estimate(Y0: np.ndarray, U: np.ndarray) -> int:
    """``s_0 = ceil(trace(Y_0^* U) / p)`` (Algorithm 4, eq. (trace)):
    for ``U = Q Y_0`` with Gaussian ``Y_0`` the expectation of the trace is
    ``p trace(Q) = p s``."""
    p = Y0.shape[1]
    return int(math.ceil(float(np.real(np.trace(Y0.conj().T @ U))) / p))


def search(solver: ShiftedSolver, w: np.ndarray, Y_pool: np.ndarray, p: int,
           alpha: float = 1.5, tau: float = 1e-3, t_max: Optional[int] = None) -> SearchResult:
    """Algorithm 4: filter ``p`` Gaussian columns, estimate ``s_0`` from the
    trace, widen the block to ``s_dagger`` columns, and repeat the
    rank-revealing QR (column-pivoted Householder QR) until the block is
    numerically rank deficient; then ``t`` is its rank and ``U_1`` the first
    ``t`` columns of ``Q``.  Columns are taken from ``Y_pool`` in order.
    ``t_max`` (default ``n``) caps ``s_dagger``; a block that is still of full
    rank at the cap raises ``ValueError``."""
    n = Y_pool.shape[0]
    cap = n if t_max is None else min(t_max, n)
    if not 1 <= p <= cap:
        raise ValueError("p out of range")
    # first filtered sample
    Y0 = Y_pool[:, :p]
    used = p
    U = apply_filter(solver, w, Y0)
    filters = 1
    # trace estimate
    s0 = trace_estimate(Y0, U)
    sd = min(max(p, s0), cap)
    rounds = 0
    while True:
        # widen the block to s_dagger columns
        if sd > p:
            if used + (sd - p) > Y_pool.shape[1]:
                raise ValueError("random column pool exhausted")
            Yt = Y_pool[:, used:used + sd - p]
            used += sd - p
            U = np.hstack([U, apply_filter(solver, w, Yt)])
            filters += 1
        else:
            sd = p
        # rank-revealing QR and rank test
        Q, R, _ = sla.qr(U, mode="economic", pivoting=True)
        rounds += 1
        t = numerical_rank(R, tau)
        if t < sd:
            return SearchResult(Q[:, :t], t, s0, rounds, used, filters)
        nxt = min(int(math.ceil(alpha * t)), cap)
        if nxt <= t:
            raise ValueError("block of full rank at the column cap")
        p, U, sd = t, Q[:, :t], nxt


def gfeast_search(A: np.ndarray, B: np.ndarray, Y_pool: np.ndarray, center: complex,
                  radius: float, N: int, p: int, alpha: float = 1.5, tau: float = 1e-3,
                  rule: int = TRAPEZOID, eps: float = 1e-10, eta: float = 1e-3,
                  max_iter: int = 20, t_max: Optional[int] = None):
    """Algorithm 5 with Algorithm 4 as its Search call: returns (Result, SearchResult)."""
    z, w = contour_nodes(center, radius, N, rule)
    solver = ShiftedSolver(A, B, z)
    sr = search(solver, w, Y_pool, p, alpha, tau, t_max)
    res = gfeast_from(A, B, sr.U1, center, radius, N, rule, eps, eta, max_iter, solver,
                      filters=sr.filters)
    return res, sr


# ---------------------------------------------------------------------------
# Derivative of the inside eigenvalues (first-order perturbation theory)
# ---------------------------------------------------------------------------

def eigenvalue_derivatives(B: np.ndarray, lam: np.ndarray, X: np.ndarray, Yl: np.ndarray,
                           dA: np.ndarray, dB: np.ndarray) -> np.ndarray:
    """``d lam_i = y_i^*(dA - lam_i dB) x_i / (y_i^* B x_i)`` for every column."""
    out = np.zeros(len(lam), dtype=np.complex128)
    for i in range(len(lam)):
        x, y = X[:, i], Yl[:, i]
        out[i] = np.vdot(y, (dA - lam[i] * dB) @ x) / np.vdot(y, B @ x)
    return out


def loss_gradient(B: np.ndarray, lam: np.ndarray, X: np.ndarray, Yl: np.ndarray):
    """Gradients of ``L = sum_i |lam_i|^2`` with respect to ``A`` and ``B``.

    With ``d lam_i = y_i^*(dA - lam_i dB) x_i / s_i``, ``s_i = y_i^* B x_i`` one has
    ``dL = sum_i 2 Re(conj(lam_i) d lam_i) = Re <G_A, dA> + Re <G_B, dB>`` where
    ``<G, D> = sum conj(G) D`` and
    ``G_A = sum_i 2 lam_i y_i x_i^* / conj(s_i)`` and
    ``G_B = -sum_i 2 |lam_i|^2 y_i x_i^* / conj(s_i)``.
    (This is the convention of PyTorch's complex autograd for a real loss.)
    """
    n = X.shape[0]
    GA = np.zeros((n, n), dtype=np.complex128)
    GB = np.zeros((n, n), dtype=np.complex128)
    for i in range(len(lam)):
        x, y = X[:, i], Yl[:, i]
        s = np.vdot(y, B @ x)
        outer = np.outer(y, x.conj()) / np.conj(s)
        GA += 2.0 * lam[i] * outer
        GB -= 2.0 * abs(lam[i]) ** 2 * outer
    return GA, GB
