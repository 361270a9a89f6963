"""Kernel-level GPU tests through the C ABI: the MFMA complex GEMM, the batched
LU with partial pivoting and the blocked triangular solves, against NumPy in
FP64 (the plain definitions of the products and of P M = L U)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_1404_1768_amd as fm  # noqa: E402

DEV = torch.device("cuda:0")


def crand(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (64, 64, 64), (130, 70, 200),
                                   (65, 129, 16), (300, 160, 1000)])
@pytest.mark.parametrize("transA", [0, 2])
@pytest.mark.parametrize("batch", [1, 3])
def test_zgemm_matches_numpy(M, N, K, transA, batch):
    rng = np.random.default_rng(M * 7 + N + K)
    A = crand(rng, batch, M, K) if transA == 0 else crand(rng, batch, K, M)
    B = crand(rng, batch, K, N)
    Cm = crand(rng, batch, M, N)
    alpha, beta = 0.7 - 0.2j, -0.3 + 1.1j
    opA = A if transA == 0 else np.conj(np.transpose(A, (0, 2, 1)))
    ref = alpha * opA @ B + beta * Cm
    tA, tB, tC = (torch.from_numpy(np.ascontiguousarray(x)).to(DEV) for x in (A, B, Cm))
    fm.zgemm_batched(tA, tB, tC, alpha, beta, transA)
    out = tC.cpu().numpy()
    scale = np.abs(alpha) * np.sqrt(K) * 2 + np.abs(beta) * 2
    assert np.max(np.abs(out - ref)) < 1e-13 * scale * max(1.0, np.sqrt(K))


def test_zgemm_beta_zero_ignores_nan_output():
    rng = np.random.default_rng(1)
    A, B = crand(rng, 1, 40, 30), crand(rng, 1, 30, 50)
    C = np.full((1, 40, 50), np.nan + 0j)
    tC = torch.from_numpy(C).to(DEV)
    fm.zgemm_batched(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), tC, 1.0, 0.0)
    assert np.allclose(tC.cpu().numpy(), A @ B, atol=1e-12)


def _apply_pivots(M, piv):
    P = M.copy()
    for i, p in enumerate(piv):
        if p != i:
            P[[i, p]] = P[[p, i]]
    return P


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130, 333, 1000])
@pytest.mark.parametrize("nb", [0, 64])
def test_zgetrf_reconstructs_and_pivots_partially(n, nb):
    rng = np.random.default_rng(n)
    batch = 3
    M = crand(rng, batch, n, n)
    tM = torch.from_numpy(M.copy()).to(DEV)
    piv, info = fm.zgetrf_batched(tM, nb=nb)
    F = tM.cpu().numpy()
    piv, info = piv.cpu().numpy(), info.cpu().numpy()
    assert np.all(info == 0)
    for b in range(batch):
        L = np.tril(F[b], -1) + np.eye(n)
        U = np.triu(F[b])
        assert np.all((piv[b] >= np.arange(n)) & (piv[b] < n))
        PM = _apply_pivots(M[b], piv[b])
        err = np.linalg.norm(PM - L @ U) / np.linalg.norm(M[b])
        assert err < 1e-14 * n, err
        # partial pivoting with the |re| + |im| measure: |l| <= |re|+|im| of the
        # pivot over |pivot| <= sqrt(2) for every multiplier
        assert np.abs(L).max() <= np.sqrt(2.0) * (1 + 1e-12)


def test_zgetrf_many_workgroups_per_panel_step():
    # batch 32 at n = 2000: each panel step launches ~1000 workgroups, more than
    # are resident at once, so workgroups of one launch start at different times
    # (a kernel that rewrites its own input in place would show here)
    rng = np.random.default_rng(7)
    n, batch = 2000, 32
    M = crand(rng, batch, n, n)
    tM = torch.from_numpy(M).to(DEV)
    piv, info = fm.zgetrf_batched(tM)
    assert np.all(info.cpu().numpy() == 0)
    F, piv = tM.cpu().numpy(), piv.cpu().numpy()
    for b in (0, batch - 1):
        L = np.tril(F[b], -1) + np.eye(n)
        U = np.triu(F[b])
        err = np.linalg.norm(_apply_pivots(M[b], piv[b]) - L @ U) / np.linalg.norm(M[b])
        assert err < 1e-14 * n, err


@pytest.mark.parametrize("n,nb", [(600, 64), (2100, 0)])
def test_zgetrf_leaf_row_blocks_past_the_last_row(n, nb):
    # the panel leaves stage their rows through LDS in fixed blocks; at these
    # orders whole blocks lie below the last row of a matrix and must be
    # skipped (the last matrix of the batch ends its allocation)
    rng = np.random.default_rng(n + 11)
    batch = 2
    M = crand(rng, batch, n, n)
    tM = torch.from_numpy(M).to(DEV)
    piv, info = fm.zgetrf_batched(tM, nb=nb)
    assert np.all(info.cpu().numpy() == 0)
    F, piv = tM.cpu().numpy(), piv.cpu().numpy()
    for b in range(batch):
        L = np.tril(F[b], -1) + np.eye(n)
        U = np.triu(F[b])
        err = np.linalg.norm(_apply_pivots(M[b], piv[b]) - L @ U) / np.linalg.norm(M[b])
        assert err < 1e-14 * n, err


def test_zgetrf_reports_exact_zero_pivot():
    n = 40
    rng = np.random.default_rng(5)
    M = crand(rng, 2, n, n)
    M[1][:, 17] = 0.0                       # column 17 of the second matrix is zero
    tM = torch.from_numpy(M).to(DEV)
    _, info = fm.zgetrf_batched(tM)
    info = info.cpu().numpy()
    assert info[0] == 0 and info[1] == 18


@pytest.mark.parametrize("n,nrhs", [(1, 1), (64, 3), (200, 37), (1000, 160)])
@pytest.mark.parametrize("trans", [0, 2])
def test_zgetrs_backward_error(n, nrhs, trans):
    rng = np.random.default_rng(n + nrhs)
    batch = 2
    M = crand(rng, batch, n, n)
    R = crand(rng, batch, n, nrhs)
    tM = torch.from_numpy(M.copy()).to(DEV)
    piv, info = fm.zgetrf_batched(tM)
    tX = torch.from_numpy(R.copy()).to(DEV)
    fm.zgetrs_batched(tM, piv, tX, trans=trans)
    X = tX.cpu().numpy()
    for b in range(batch):
        Mb = M[b] if trans == 0 else M[b].conj().T
        be = np.linalg.norm(Mb @ X[b] - R[b]) / (np.linalg.norm(Mb) * np.linalg.norm(X[b]) + np.linalg.norm(R[b]))
        assert be < 1e-15 * n + 1e-15, be
