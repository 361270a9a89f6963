"""Seeded synthetic pencils and start blocks for the oblique-projection FEAST path.

This module builds inputs only: it holds none of the method's arithmetic and is
shared, as the one common dependency, by the CPU oracle (``oracle/``) and by the
GPU path's tests and benchmark.

Construction (the test problems are synthetic stand-ins for the Matrix Market
pencils of Table 1, which are not available here):

* ``A = P D Q`` and ``B = P Q`` with ``P, Q = I + c G``.  This is a Weierstrass
  form (Theorem 2.1) with ``T = P^{-1}`` and ``S = Q^{-1}``: the eigenvalues of
  the pencil are exactly the diagonal of ``D`` and the right eigenvector of
  ``d_i`` is column ``i`` of ``Q^{-1}``.
* ``G`` has i.i.d. complex Gaussian entries of variance ``g_var`` (default
  ``1/n``, so ``c G`` is a small perturbation of the identity; ``g_var = 1`` is
  the literal unit-variance reading, kept for stress runs).
* Eigenvalue positions are area-uniform in a disk or an annulus around the
  contour centre.
* The start block ``V`` is complex Gaussian with ``E|v|^2 = 1``.

Seeds: ``numpy.random.SeedSequence(14041768 + k)`` for workload ``k``; the
children are spawned in the fixed order ``[G_P, G_Q, D_inside, D_outside,
D_cluster, V]``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 14041768


@dataclasses.dataclass
class Pencil:
    """One synthetic pencil (row-major complex128 arrays)."""

    A: np.ndarray          # n x n
    B: np.ndarray          # n x n
    V: np.ndarray          # n x m start block
    d: np.ndarray          # n exact eigenvalues (diagonal of D)
    P: np.ndarray          # n x n
    Q: np.ndarray          # n x n
    center: complex        # contour centre gamma
    radius: float          # contour radius rho
    nodes: int             # quadrature nodes N
    m: int                 # subspace size t
    name: str = ""

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def inside_mask(self) -> np.ndarray:
        return np.abs(self.d - self.center) < self.radius

    @property
    def s(self) -> int:
        """Exact number of eigenvalues strictly inside the circle."""
        return int(np.count_nonzero(self.inside_mask))


def _cgauss(rng: np.random.Generator, shape, var: float) -> np.ndarray:
    sd = math.sqrt(var / 2.0)
    return rng.normal(0.0, sd, shape) + 1j * rng.normal(0.0, sd, shape)


def _area_uniform(rng: np.random.Generator, count: int, r1: float, r2: float,
                  center: complex) -> np.ndarray:
    """``count`` points area-uniform in the annulus ``r1 <= |z - center| < r2``."""
    if count == 0:
        return np.zeros(0, dtype=np.complex128)
    u = rng.random(count)
    th = 2.0 * math.pi * rng.random(count)
    r = np.sqrt(r1 * r1 + u * (r2 * r2 - r1 * r1))
    return center + r * np.exp(1j * th)


def make_pencil(n: int, m: int, inside: int, inside_radius: float,
                outside_r: tuple, center: complex = 0.0, radius: float = 1.0,
                nodes: int = 16, c: float = 0.05, cluster: int = 0,
                cluster_r: tuple = (1.05, 1.2), g_var: Optional[float] = None,
                seed: int = BASE_SEED, name: str = "") -> Pencil:
    """Build ``A = P D Q``, ``B = P Q`` and a start block ``V`` (n x m).

    ``inside`` eigenvalues are area-uniform in ``|z - center| < inside_radius``,
    ``cluster`` in the annulus ``cluster_r`` and the remaining
    ``n - inside - cluster`` in the annulus ``outside_r`` (radii relative to the
    centre).
    """
    if g_var is None:
        g_var = 1.0 / n
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(6)
    rgp, rgq, rdi, rdo, rdc, rv = [np.random.default_rng(k) for k in kids]
    G_P = _cgauss(rgp, (n, n), g_var)
    G_Q = _cgauss(rgq, (n, n), g_var)
    outside = n - inside - cluster
    if outside < 0:
        raise ValueError("inside + cluster exceeds n")
    d = np.concatenate([
        _area_uniform(rdi, inside, 0.0, inside_radius, center),
        _area_uniform(rdo, outside, outside_r[0], outside_r[1], center),
        _area_uniform(rdc, cluster, cluster_r[0], cluster_r[1], center),
    ])
    V = _cgauss(rv, (n, m), 1.0)
    eye = np.eye(n, dtype=np.complex128)
    P = eye + c * G_P
    Q = eye + c * G_Q
    B = P @ Q
    A = (P * d[None, :]) @ Q
    return Pencil(A=np.ascontiguousarray(A), B=np.ascontiguousarray(B),
                  V=np.ascontiguousarray(V), d=d, P=P, Q=Q,
                  center=complex(center), radius=float(radius), nodes=nodes,
                  m=m, name=name)


# ---------------------------------------------------------------------------
# The five workloads.  Index k selects seed BASE_SEED + k.
# ---------------------------------------------------------------------------

def workload(k: int, g_var: Optional[float] = None, n_override: Optional[int] = None) -> Pencil:
    """Workloads 1, 2, 3 and 5 (single pencils); see ``batch_workload`` for 4.

    ``n_override`` shrinks a workload to a smaller order with the same recipe
    (eigenvalue fractions kept), for quick tests.
    """
    seed = BASE_SEED + k
    if k == 1:
        n = n_override or 200
        s = max(1, round(20 * n / 200))
        return make_pencil(n, m=max(s + 10, round(30 * n / 200)), inside=s, inside_radius=0.8,
                           outside_r=(1.5, 5.0), center=0.0, radius=1.0, nodes=16,
                           c=0.1, g_var=g_var, seed=seed, name="plain-n%d" % n)
    if k == 2:
        n = n_override or 4000
        s = max(1, round(100 * n / 4000))
        m = max(s + 8, round(160 * n / 4000))
        return make_pencil(n, m=m, inside=s, inside_radius=0.9, outside_r=(1.3, 10.0),
                           center=1 + 1j, radius=1.0, nodes=32, c=0.05,
                           g_var=g_var, seed=seed, name="fp64-n%d" % n)
    if k == 3:
        n = n_override or 8000
        s = max(1, round(120 * n / 8000))
        m = max(s + 8, round(256 * n / 8000))
        rest = n - s
        cluster = int(round(0.05 * rest))
        return make_pencil(n, m=m, inside=s, inside_radius=1.0, outside_r=(1.2, 20.0),
                           center=0.0, radius=1.0, nodes=32, c=0.05, cluster=cluster,
                           cluster_r=(1.05, 1.2), g_var=g_var, seed=seed,
                           name="mixed-n%d" % n)
    if k == 5:
        n = n_override or 2048
        s = max(1, round(40 * n / 2048))
        m = max(s + 8, round(64 * n / 2048))
        return make_pencil(n, m=m, inside=s, inside_radius=0.9, outside_r=(1.3, 10.0),
                           center=0.0, radius=1.0, nodes=32, c=0.05, g_var=g_var,
                           seed=seed, name="adjoint-n%d" % n)
    raise ValueError("workload %r is not a single pencil" % (k,))


def batch_sizes(count: int = 64, lo: int = 256, hi: int = 2048, seed: int = BASE_SEED + 4):
    """Orders n_p ~ U[lo, hi] and centres gamma_p ~ U([-2,2]^2) of the batch workload."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    ns = rng.integers(lo, hi + 1, size=count)
    centers = rng.uniform(-2.0, 2.0, size=count) + 1j * rng.uniform(-2.0, 2.0, size=count)
    return [int(x) for x in ns], [complex(x) for x in centers]


def batch_workload(count: int = 64, lo: int = 256, hi: int = 2048, nodes: int = 16):
    """Workload 4: ``count`` independent pencils of uneven order.

    Pencil p has ``floor(n_p/20)`` eigenvalues in ``|z - gamma_p| < 0.9``, the rest
    in the annulus 1.3..10 about gamma_p, ``m_p = 2 floor(n_p/20)``, radius 1.
    """
    ns, centers = batch_sizes(count, lo, hi)
    out = []
    for p, (n, g) in enumerate(zip(ns, centers)):
        s = max(1, n // 20)
        out.append(make_pencil(n, m=2 * s, inside=s, inside_radius=0.9,
                               outside_r=(1.3, 10.0), center=g, radius=1.0, nodes=nodes,
                               c=0.05, seed=BASE_SEED + 4 + 1000 * (p + 1),
                               name="batch-%d-n%d" % (p, n)))
    return out


def start_block(n: int, m: int, seed: int) -> np.ndarray:
    """Complex Gaussian n x m block with unit-variance entries."""
    return _cgauss(np.random.default_rng(seed), (n, m), 1.0)


def pencil_from_eigenvalues(d: np.ndarray, m: int, center: complex, radius: float, nodes: int,
                            c: float = 0.05, seed: int = BASE_SEED, name: str = "") -> Pencil:
    """``A = P D Q``, ``B = P Q`` with the given eigenvalues ``d`` (same P, Q and V
    recipe as ``make_pencil``; children ``[G_P, G_Q, V]`` of the seed)."""
    d = np.asarray(d, dtype=np.complex128)
    n = d.size
    rgp, rgq, rv = (np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(3))
    eye = np.eye(n, dtype=np.complex128)
    P = eye + c * _cgauss(rgp, (n, n), 1.0 / n)
    Q = eye + c * _cgauss(rgq, (n, n), 1.0 / n)
    B = P @ Q
    A = (P * d[None, :]) @ Q
    V = _cgauss(rv, (n, m), 1.0)
    return Pencil(A=np.ascontiguousarray(A), B=np.ascontiguousarray(B), V=np.ascontiguousarray(V),
                  d=d, P=P, Q=Q, center=complex(center), radius=float(radius), nodes=nodes, m=m,
                  name=name)


# L-shaped region: the unit square [-1, 1]^2 without its upper-right quarter
L_REGION = np.array([-1 - 1j, 1 - 1j, 1 + 0j, 0 + 0j, 0 + 1j, -1 + 1j], dtype=np.complex128)


def region_workload(n: int = 600, inside: int = 30, notch: int = 8, nodes: int = 32,
                    seed: int = BASE_SEED + 6):
    """An irregular region (the L-shaped polygon ``L_REGION``): ``inside``
    eigenvalues uniform in the L, ``notch`` in the cut-out quarter
    ``(0.15, 0.85)^2`` (inside the enclosing circle, outside the region) and the
    rest area-uniform in ``2.5 <= |z| < 8``.  Returns the pencil (its circle
    fields are placeholders: the driver derives the circle from the region)
    and the mask of the eigenvalues inside the region."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    pts = []
    while len(pts) < inside:
        x, y = rng.uniform(-0.95, 0.95, size=2)
        if x <= -0.05 or y <= -0.05:               # the L, clear of its inner edges
            pts.append(x + 1j * y)
    notch_pts = rng.uniform(0.15, 0.85, size=notch) + 1j * rng.uniform(0.15, 0.85, size=notch)
    out = _area_uniform(rng, n - inside - notch, 2.5, 8.0, 0.0)
    d = np.concatenate([np.array(pts), notch_pts, out])
    p = pencil_from_eigenvalues(d, m=2 * (inside + notch), center=0.0, radius=1.0, nodes=nodes,
                                seed=seed + 1, name="region-L-n%d" % n)
    mask = np.zeros(n, dtype=bool)
    mask[:inside] = True
    return p, mask


# Table 1 of the paper: (name, n, nnz(A), nnz(B), property of A, property of B).
# The Matrix Market files are not available; these are the shapes the
# stand-ins below reproduce.
TABLE1 = [
    ("BFW398", 398, 3678, 2910, "unsym", "symind"),
    ("BFW782", 782, 7514, 5982, "unsym", "symind"),
    ("PLAT/PLSK1919", 1919, 17159, 4831, "symind", "skew"),
    ("BCSSTK/M13", 2003, 42943, 11973, "spd", "spsd"),
    ("BCSSTK/M27", 1224, 28675, 28675, "spd", "symind"),
    ("MHD3200", 3200, 68026, 18316, "unsym", "symind"),
    ("MHD4800", 4800, 102252, 27520, "unsym", "symind"),
]


def _pattern(rng, n: int, k: int, band: Optional[int], upper: bool = False):
    """``k`` random positions (i, j) anywhere (repeats possible), or, with
    ``band``, ``k`` distinct off-diagonal positions with ``|i - j| <= band``
    (``upper``: ``0 < j - i <= band``)."""
    if band is None:
        i = rng.integers(0, n, k)
        return i, rng.integers(0, n, k)
    offs = np.arange(1, band + 1)
    if not upper:
        offs = np.concatenate([-offs[::-1], offs])
    ci = np.repeat(np.arange(n), offs.size)
    cj = ci + np.tile(offs, n)
    ok = (cj >= 0) & (cj < n)
    ci, cj = ci[ok], cj[ok]
    sel = rng.choice(ci.size, min(k, ci.size), replace=False)
    return ci[sel], cj[sel]


def _sparse_real(rng, n: int, nnz: int, kind: str, band: Optional[int] = None) -> np.ndarray:
    """A dense array holding a real sparse matrix with about ``nnz`` non-zeros
    of the given structure: unsym, symind (symmetric indefinite), skew,
    spd (symmetric, diagonally dominant, positive diagonal), spsd (as spd with
    a tenth of the rows and columns zero, hence singular).  ``band``: the
    off-diagonal non-zeros lie within that distance of the diagonal (else
    anywhere)."""
    M = np.zeros((n, n))
    if kind == "unsym":
        k = max(nnz - n, 0)
        i, j = _pattern(rng, n, k, band)
        M[i, j] = rng.normal(size=k)
        M[np.arange(n), np.arange(n)] += rng.normal(size=n) + 2.0 * rng.choice([-1, 1], n)
        return M
    off = nnz - (0 if kind == "skew" else n)
    if kind == "spsd":  # the zeroed tenth of the rows and columns removes about 19%
        off = int(off / 0.81)
    half = max(off // 2, 0)
    i, j = _pattern(rng, n, half, band, upper=True)
    keep = i != j
    i, j = np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])
    U = np.zeros((n, n))
    U[i, j] = rng.normal(size=i.size)  # strict upper triangle
    if kind == "skew":
        return U - U.T
    M = U + U.T
    if kind == "symind":
        M[np.arange(n), np.arange(n)] = rng.normal(size=n) * 2.0
    else:  # spd / spsd: diagonally dominant
        M[np.arange(n), np.arange(n)] = np.abs(M).sum(axis=1) + 1.0
        if kind == "spsd":
            z = rng.choice(n, n // 10, replace=False)
            M[z, :] = 0.0
            M[:, z] = 0.0
    return M


def sparse_standin(k: int, m: int = 40, seed: int = BASE_SEED + 100, banded: bool = False):
    """Stand-in for problem k (1..7) of Table 1: real A, B of its order, number
    of non-zeros and structure (random values and pattern), returned dense as
    complex128, with a complex Gaussian start block V (n x m).  ``banded``:
    the off-diagonal non-zeros of both lie within a band of half-width
    ``ceil(nnz_A / n)`` around the diagonal instead of anywhere."""
    name, n, nnz_a, nnz_b, ka, kb = TABLE1[k - 1]
    ra, rb, rv = (np.random.default_rng(s) for s in np.random.SeedSequence(seed + k).spawn(3))
    band = int(math.ceil(nnz_a / n)) if banded else None
    A = _sparse_real(ra, n, nnz_a, ka, band).astype(np.complex128)
    B = _sparse_real(rb, n, nnz_b, kb, band).astype(np.complex128)
    V = _cgauss(rv, (n, m), 1.0)
    return name, A, B, V
