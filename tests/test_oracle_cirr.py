"""Pins of the oracle's Block_CIRR (Algorithm 1).

For ``A = P D Q``, ``B = P Q``: ``(zB - A)^{-1} = Q^{-1} (zI - D)^{-1} P^{-1}``, and
the half-offset trapezoid rule turns ``sum_j w_j mu_j^i / (z_j - d)`` into
``mu(d)^i / (1 + mu(d)^N)`` for ``0 <= i < N`` (partial fractions of that
rational function), so the discrete moments have a closed form."""
import numpy as np
import pytest

import pencilgen as pg
from oracle import gfeast as o


def _pencil(n=120, inside=9, outside_r=(4.0, 10.0), seed=41):
    return pg.make_pencil(n, m=24, inside=inside, inside_radius=0.8, outside_r=outside_r,
                          center=-0.4 + 0.7j, radius=1.2, nodes=32, c=0.05, seed=seed, name="cirr")


@pytest.mark.parametrize("g", [1, 3, 5])
def test_moments_closed_form(g):
    p = _pencil()
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    Y = p.V[:, :4]
    M = o.cirr_moments(o.ShiftedSolver(p.A, p.B, z), z, w, Y, g, p.center, p.radius)
    mu = (p.d - p.center) / p.radius
    for i in range(g):
        f = mu ** i / (1.0 + mu ** p.nodes)
        ref = np.linalg.solve(p.Q, f[:, None] * np.linalg.solve(p.P, Y))
        assert np.max(np.abs(M[:, 4 * i:4 * (i + 1)] - ref)) < 1e-12 * np.abs(ref).max()


def test_block_cirr_finds_the_planted_spectrum():
    p = _pencil()
    r = o.block_cirr(p.A, p.B, p.V[:, :4], 4, p.center, p.radius, p.nodes)
    assert r.t == 16
    got, ref = np.sort_complex(r.lam), np.sort_complex(p.d[p.inside_mask])
    assert len(got) == len(ref) == 9
    assert np.max(np.abs(got - ref)) < 1e-10
    assert np.all(r.r < 1e-10)
    # the moment block has numerical rank s: h g - s singular values at rounding level
    assert r.sv[8] > 1e-6 * r.sv[0] and r.sv[9] < 1e-10 * r.sv[0]


def test_block_cirr_is_basis_invariant():
    # Rayleigh-Ritz depends on the span only: any orthonormal basis of the moment
    # block gives the eigenvalues of the SVD's U (the GPU path uses Cholesky QR)
    p = _pencil()
    z, w = o.contour_nodes(p.center, p.radius, p.nodes)
    M = o.cirr_moments(o.ShiftedSolver(p.A, p.B, z), z, w, p.V[:, :3], 4, p.center, p.radius)
    Qm, _ = np.linalg.qr(M)
    U, _, _ = np.linalg.svd(M, full_matrices=False)
    ev = []
    for W in (Qm, U):
        a, b, _ = o.reduced_eig(W.conj().T @ p.A @ W, W.conj().T @ p.B @ W)
        lam = o.eigenvalues_from(a, b)
        ev.append(np.sort_complex(lam[o.inside(lam, p.center, p.radius)]))
    # (the three rounding-level directions of this rank-9 block give spurious
    # Ritz values too, identical in both bases; the final residual test drops them)
    assert len(ev[0]) == len(ev[1]) and np.max(np.abs(ev[0] - ev[1])) < 1e-10


def test_block_cirr_with_too_small_a_block_misses_eigenvalues():
    # h g < s: the Ritz space cannot hold the s eigenvectors (Algorithm 1 needs t >= s)
    p = _pencil()
    r = o.block_cirr(p.A, p.B, p.V[:, :2], 2, p.center, p.radius, p.nodes)
    assert r.t == 4 and len(r.lam) < 9
