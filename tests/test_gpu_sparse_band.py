"""Algorithm 5 on sparse pencils in CSR form (feast_solve_csr): reverse
Cuthill-McKee ordering on the host, band LU of every node and band solves on
the GPU.  The problems are the banded variants of the Table 1 stand-ins
(non-zeros within ceil(nnz(A)/n) of the diagonal); their reference eigenvalues
inside each circle come from the oracle's dense spectrum
(tests/golden/standin_banded_contours.json), and the oracle's own Algorithm 5
runs on the small ones.  Closed forms pin the degenerate bands (diagonal and
tridiagonal Toeplitz pencils)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linear_sum_assignment

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_1404_1768_amd as fm  # noqa: E402
import pencilgen as pg  # noqa: E402
from oracle import gfeast as o  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "standin_banded_contours.json")


def _csr(M):
    S = sp.csr_matrix(M)
    S.sort_indices()
    return (torch.from_numpy(S.indptr.astype(np.int32)).to("cuda"),
            torch.from_numpy(S.indices.astype(np.int32)).to("cuda"),
            torch.from_numpy(S.data.astype(np.complex128)).to("cuda"))


def _case(k):
    with open(GOLDEN) as f:
        g = json.load(f)[str(k)]
    name, A, B, V = pg.sparse_standin(k, banded=True)
    ref = np.array([complex(*z) for z in g["inside"]])
    return A, B, V, complex(*g["center"]), g["radius"], ref


def _match(a, b):
    D = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(D)
    return D[r, c].max()


def _residuals(A, B, X, lam):
    AX, BX = A @ X, B @ X
    return np.linalg.norm(AX - BX * lam, axis=0) / (np.linalg.norm(AX, axis=0) +
                                                     np.linalg.norm(BX, axis=0))


def _solve_csr(A, B, V, c, r, nodes=16, rule=fm.GAUSS_LEGENDRE):
    n, m = A.shape[0], V.shape[1]
    dV = torch.from_numpy(np.ascontiguousarray(V)).to("cuda")
    with fm.Plan(n, m, c, r, nodes, rule=rule, eps=1e-10, prec=fm.FP64) as plan:
        return plan.solve_csr(_csr(A), _csr(B), dV)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_banded_standin_eigenvalues(k):
    A, B, V, c, r, ref = _case(k)
    res = _solve_csr(A, B, V, c, r)
    kl, ku = res.band
    assert kl + ku <= 63
    assert res.flag == 1 and res.err <= 1e-10
    assert len(res.lam) == len(ref)
    scale = max(1.0, abs(c) + r)
    assert _match(res.lam, ref) <= 1e-8 * scale
    assert np.all(_residuals(A, B, res.X.cpu().numpy(), res.lam) <= 1e-10)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_banded_standin_matches_oracle_and_dense_path(k):
    """The oracle's Algorithm 5 (dense) and the GPU's dense path find the same
    eigenvalues, with the same residual history, as the sparse path.  (k = 4:
    B singular, infinite eigenvalues mapped to zero by the filter.)"""
    A, B, V, c, r, ref = _case(k)
    res = _solve_csr(A, B, V, c, r)
    ro = o.gfeast(A, B, V, c, r, 16, rule=o.GAUSS_LEGENDRE)
    assert ro.flag == 1 and len(ro.lam) == len(res.lam)
    scale = max(1.0, abs(c) + r)
    assert _match(res.lam, ro.lam) <= 1e-8 * scale
    assert res.iters == ro.iters
    n, m = A.shape[0], V.shape[1]
    dA, dB, dV = (torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in (A, B, V))
    with fm.Plan(n, m, c, r, 16, rule=fm.GAUSS_LEGENDRE, eps=1e-10, prec=fm.FP64) as plan:
        rd = plan.solve(dA, dB, dV)
    assert rd.iters == res.iters and len(rd.lam) == len(res.lam)
    assert _match(res.lam, rd.lam) <= 1e-9 * scale
    # e(k) of every iteration agrees while it is above the rounding floor
    for e1, e2 in zip(res.errs, rd.errs):
        if max(e1, e2) > 1e-12:
            assert abs(e1 - e2) <= 1e-3 * max(e1, e2)


def test_scrambled_pencil_same_eigenpairs():
    """A symmetric permutation of the pencil (as a sparse pencil arrives in an
    arbitrary order): the ordering recovers a narrow band, the eigenvalues are
    unchanged and the eigenvectors come back in the caller's row order."""
    A, B, V, c, r, ref = _case(3)
    n = A.shape[0]
    q = np.random.default_rng(77).permutation(n)
    As, Bs, Vs = A[np.ix_(q, q)], B[np.ix_(q, q)], V[q]
    r0 = _solve_csr(A, B, V, c, r)
    r1 = _solve_csr(As, Bs, Vs, c, r)
    assert r1.band[0] + r1.band[1] <= 63
    assert r1.flag == 1 and len(r1.lam) == len(r0.lam)
    assert _match(r1.lam, r0.lam) <= 1e-9
    X0, X1 = r0.X.cpu().numpy(), r1.X.cpu().numpy()
    assert np.all(_residuals(As, Bs, X1, r1.lam) <= 1e-10)
    # eigenvector of the same eigenvalue: X1 = X0[q] (both unit norm with the
    # largest-modulus entry real positive, a normalisation rows do not change)
    D = np.abs(r0.lam[:, None] - r1.lam[None, :])
    i0, i1 = linear_sum_assignment(D)
    for a, b in zip(i0, i1):
        assert np.abs(X1[:, b] - X0[q, a]).max() <= 1e-8


def test_one_plan_reuses_the_ordering_not_the_values():
    """One plan, four calls: the pencil, the same pattern with A scaled by
    1.001 (the ordering is reused; the values and factors are not: the
    eigenvalues scale with A), a symmetric permutation (a new pattern, ordered
    afresh) and the first pencil again (ordered again, same result)."""
    A, B, V, c, r, ref = _case(3)
    n, m = A.shape[0], V.shape[1]
    q = np.random.default_rng(5).permutation(n)
    calls = [(A, B, V), (A * 1.001, B, V), (A[np.ix_(q, q)], B[np.ix_(q, q)], V[q]), (A, B, V)]
    out = []
    with fm.Plan(n, m, c, r, 16, rule=fm.GAUSS_LEGENDRE, eps=1e-10, prec=fm.FP64) as plan:
        for Ak, Bk, Vk in calls:
            dV = torch.from_numpy(np.ascontiguousarray(Vk)).to("cuda")
            out.append(plan.solve_csr(_csr(Ak), _csr(Bk), dV))
    r0, r1, r2, r3 = out
    scale = max(1.0, abs(c) + r)
    assert r0.flag == 1 and len(r0.lam) == len(ref)
    assert len(r1.lam) == len(r0.lam) and _match(r1.lam, 1.001 * r0.lam) <= 1e-8 * scale
    assert _match(r1.lam, r0.lam) > 1e-6 * scale  # not the first call's values
    assert len(r2.lam) == len(r0.lam) and _match(r2.lam, r0.lam) <= 1e-9 * scale
    assert r3.band == r0.band and _match(r3.lam, r0.lam) <= 1e-12 * scale


def _wide_band_pencil(n, kl, ku, seed):
    """A full random band (kl below, ku above the diagonal) on a spread
    diagonal: eigenvalue condition numbers stay below about 12, and z B - A
    on the contour pivots on about a fifth of its columns, anywhere in the
    kl rows below the diagonal."""
    rng = np.random.default_rng(seed)
    i, j = np.indices((n, n))
    band = (j - i <= ku) & (i - j <= kl)
    N1 = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    N2 = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    d = np.linspace(-4, 4, n) + 0.05j * rng.normal(size=n)
    A = np.where(band, 0.02 * N1, 0) + np.diag(d)
    B = np.where(band, 0.002 * N2, 0) + np.eye(n)
    return A.astype(np.complex128), B.astype(np.complex128)


@pytest.mark.parametrize("kl,ku", [(62, 1), (1, 62), (47, 16), (16, 47), (31, 31), (23, 8),
                                   (8, 15)])
def test_wide_bands_every_window_class(kl, ku):
    """Bands up to kl + ku = 63 in the natural order, so that every register
    window class of the band LU and the forward solve (kl + 1 up to 16, 24,
    32, 48, 64 rows) and of the backward solve (kl + ku up to 24, 32, 64) runs:
    the eigenvalues inside the circle are those of the dense spectrum and of
    the dense path."""
    import scipy.linalg as sl
    n = 480
    A, B = _wide_band_pencil(n, kl, ku, 1000 + 64 * kl + ku)
    lam = sl.eigvals(A, B)
    c = lam[np.argmin(np.abs(lam - 0.3))]
    dist = np.sort(np.abs(lam - c))
    r = 0.5 * (dist[9] + dist[10])
    inside = lam[np.abs(lam - c) < r]
    V = np.random.default_rng(3).normal(size=(n, 2 * len(inside) + 4)).astype(np.complex128)
    res = _solve_csr(A, B, V, c, r)
    assert res.band == (kl, ku)
    assert res.flag == 1 and len(res.lam) == len(inside)
    scale = max(1.0, abs(c) + r)
    assert _match(res.lam, inside) <= 1e-8 * scale
    dA, dB, dV = (torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in (A, B, V))
    with fm.Plan(n, V.shape[1], c, r, 16, rule=fm.GAUSS_LEGENDRE, eps=1e-10,
                 prec=fm.FP64) as plan:
        rd = plan.solve(dA, dB, dV)
    assert len(rd.lam) == len(res.lam) and _match(res.lam, rd.lam) <= 1e-9 * scale
    X = res.X.cpu().numpy()
    assert np.all(_residuals(A, B, X, res.lam) <= 1e-9)


@pytest.mark.parametrize("n,kl,ku", [(24, 5, 9), (7, 6, 0), (31, 2, 3)])
def test_pencils_smaller_than_one_chunk(n, kl, ku):
    """Orders below one staging chunk (32 rows) and, for n = 7, a window that
    covers the whole matrix; m below the 16 columns of a solve block."""
    import scipy.linalg as sl
    A, B = _wide_band_pencil(n, kl, ku, 77)
    lam = sl.eigvals(A, B)
    c = lam[np.argmin(np.abs(lam - 0.3))]
    dist = np.sort(np.abs(lam - c))
    r = 0.5 * (dist[2] + dist[3])
    inside = lam[np.abs(lam - c) < r]
    V = np.random.default_rng(3).normal(size=(n, min(n, 2 * len(inside) + 2))).astype(
        np.complex128)
    res = _solve_csr(A, B, V, c, r)
    assert res.band == (kl, ku)
    assert res.flag == 1 and len(res.lam) == len(inside) == 3
    scale = max(1.0, abs(c) + r)
    assert _match(res.lam, inside) <= 1e-10 * scale
    assert np.all(_residuals(A, B, res.X.cpu().numpy(), res.lam) <= 1e-10)


def test_diagonal_pencil_closed_form():
    """kl = ku = 0: A = diag(d), B = I has eigenvalues d exactly."""
    n = 600
    rng = np.random.default_rng(5)
    d = np.exp(2j * np.pi * rng.random(n)) * (1.3 + 3.0 * rng.random(n))
    d[:25] = 0.7 * np.sqrt(rng.random(25)) * np.exp(2j * np.pi * rng.random(25))
    A, B = np.diag(d), np.eye(n, dtype=np.complex128)
    V = rng.normal(size=(n, 40)) + 1j * rng.normal(size=(n, 40))
    res = _solve_csr(A, B, V, 0.0, 1.0, nodes=32, rule=fm.TRAPEZOID)
    assert res.band == (0, 0)
    inside = d[np.abs(d) < 1.0]
    assert res.flag == 1 and len(res.lam) == len(inside)
    assert _match(res.lam, inside) <= 1e-12


def test_tridiagonal_toeplitz_closed_form():
    """kl = ku = 1: A = tridiag(b, a, c), B = I has the eigenvalues
    a + 2 sqrt(b c) cos(k pi / (n + 1)), k = 1..n (b = c: a normal matrix, so
    the closed form is also what rounding leaves of them)."""
    n, a, b, cc = 300, 0.3 + 0.1j, 0.45, 0.45
    A = (np.diag(np.full(n, a)) + np.diag(np.full(n - 1, b), -1) +
         np.diag(np.full(n - 1, cc), 1)).astype(np.complex128)
    B = np.eye(n, dtype=np.complex128)
    lam = a + 2 * np.sqrt(b * cc) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    # (16 nodes and a spectrum spacing of about 0.007: far more eigenvalues
    # than the m columns keep filter values above rounding, so the filtered
    # block has full rank)
    center, radius = complex(a.real + 0.6, a.imag), 0.05
    inside = lam[np.abs(lam - center) < radius]
    V = np.random.default_rng(9).normal(size=(n, 2 * len(inside) + 4)).astype(np.complex128)
    res = _solve_csr(A, B, V, center, radius, nodes=16, rule=fm.TRAPEZOID)
    assert res.band == (1, 1)
    assert res.flag == 1 and len(res.lam) == len(inside)
    assert _match(res.lam, inside) <= 1e-11


def test_sparse_error_paths():
    A, B, V, c, r, _ = _case(1)
    n, m = A.shape[0], V.shape[1]
    dV = torch.from_numpy(np.ascontiguousarray(V)).to("cuda")
    # band factors are FP64 only
    with fm.Plan(n, m, c, r, 16, rule=fm.GAUSS_LEGENDRE, prec=fm.MIXED) as plan:
        with pytest.raises(fm.FeastError) as e:
            plan.solve_csr(_csr(A), _csr(B), dV)
        assert e.value.code == fm.FEAST_EINVAL
    # a random pattern fills the band: refused with a pointer to the dense path
    name, Aw, Bw, Vw = pg.sparse_standin(1)
    with fm.Plan(n, m, c, r, 16, rule=fm.GAUSS_LEGENDRE, prec=fm.FP64) as plan:
        with pytest.raises(fm.FeastError) as e:
            plan.solve_csr(_csr(Aw), _csr(Bw), dV)
        assert e.value.code == fm.FEAST_EINVAL and "band too wide" in str(e.value)
        # a column index out of range
        rp, ci, va = _csr(A)
        bad = ci.clone()
        bad[3] = n + 5
        with pytest.raises(fm.FeastError) as e:
            plan.solve_csr((rp, bad, va), _csr(B), dV)
        assert e.value.code == fm.FEAST_EINVAL and "out of range" in str(e.value)
        # the plan still works after the refusals
        res = plan.solve_csr(_csr(A), _csr(B), dV)
        assert res.flag == 1
