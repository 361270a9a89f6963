"""Algorithm 5 on sparse-shaped stand-ins of Table 1 (Section 5), held dense:
the Gauss-Legendre rule with 16 nodes and a 40-column subspace, as in the
paper's runs.  The eigenvalues found inside each stored circle are the dense
reference ones (tests/golden/standin_contours.json, written by the oracle), the
residuals meet the tolerance, and the oracle's own Algorithm 5 agrees."""
import json
import os

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_1404_1768_amd as fm  # noqa: E402
import pencilgen as pg  # noqa: E402
from oracle import gfeast as o  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "standin_contours.json")


def _case(k):
    with open(GOLDEN) as f:
        g = json.load(f)[str(k)]
    name, A, B, V = pg.sparse_standin(k)
    ref = np.array([complex(*z) for z in g["inside"]])
    return A, B, V, complex(*g["center"]), g["radius"], ref


def _match(a, b):
    """Largest distance of the optimal one-to-one matching of two sets (real
    pencils have conjugate pairs whose order a sort does not fix)."""
    D = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(D)
    return D[r, c].max()


def _residuals(A, B, X, lam):
    AX, BX = A @ X, B @ X
    return np.linalg.norm(AX - BX * lam, axis=0) / (np.linalg.norm(AX, axis=0) +
                                                     np.linalg.norm(BX, axis=0))


@pytest.mark.parametrize("k,prec", [(1, fm.FP64), (1, fm.MIXED), (5, fm.FP64), (2, fm.MIXED),
                                    (4, fm.FP64), (4, fm.MIXED)])
def test_standin_eigenvalues_inside_the_circle(k, prec):
    A, B, V, c, r, ref = _case(k)
    n, m = A.shape[0], V.shape[1]
    dA, dB, dV = (torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in (A, B, V))
    with fm.Plan(n, m, c, r, 16, rule=fm.GAUSS_LEGENDRE, eps=1e-10, prec=prec) as plan:
        res = plan.solve(dA, dB, dV)
    assert res.flag == 1 and res.err <= 1e-10
    assert len(res.lam) == len(ref)
    # the random pencils are not normal: eigenvalue errors reach ~1e-10 at
    # residual 1e-12 (the dense QZ and the oracle differ by as much)
    scale = max(1.0, abs(c) + r)
    assert _match(res.lam, ref) <= 1e-8 * scale
    assert np.all(_residuals(A, B, res.X.cpu().numpy(), res.lam) <= 1e-10)
    if k in (1, 4):
        # k = 4: B is singular (a tenth of its rows and columns are zero), the
        # pencil has infinite eigenvalues, which the filter maps to zero
        ro = o.gfeast(A, B, V, c, r, 16, rule=o.GAUSS_LEGENDRE)
        assert ro.flag == 1 and len(ro.lam) == len(ref)
        assert _match(res.lam, ro.lam) <= 1e-8 * scale
