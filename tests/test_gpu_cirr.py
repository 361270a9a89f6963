"""Block_CIRR (Algorithm 1) on the GPU against the oracle's Block_CIRR on the
same inputs (eigenvalues, eigenvectors, residuals) and against the planted
spectrum; the full-size run is the paper's comparison method on the metric
pencil."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_1404_1768_amd as fm  # noqa: E402
import pencilgen as pg  # noqa: E402
from oracle import gfeast as o  # noqa: E402


def to_dev(*xs):
    return [torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in xs]


def _match(a, b):
    from scipy.optimize import linear_sum_assignment
    C = np.abs(a[:, None] - b[None, :])
    i, j = linear_sum_assignment(C)
    return i, j, C[i, j]


@pytest.mark.parametrize("prec", [fm.FP64, fm.MIXED])
@pytest.mark.parametrize("h,g", [(4, 4), (3, 6)])
def test_cirr_matches_oracle(prec, h, g):
    p = pg.make_pencil(300, m=32, inside=10, inside_radius=0.8, outside_r=(2.0, 9.0),
                       center=0.5 - 0.3j, radius=1.1, nodes=32, c=0.05, seed=61, name="cirr")
    Y = p.V[:, :h]
    ref = o.block_cirr(p.A, p.B, Y, g, p.center, p.radius, p.nodes)
    A, B, Yd = to_dev(p.A, p.B, Y)
    with fm.Plan(p.n, 32, p.center, p.radius, p.nodes, prec=prec) as plan:
        lam, X, res, info = plan.cirr(A, B, Yd, g)
    assert info["t"] == h * g
    assert len(lam) == len(ref.lam) == p.s == 10
    i, j, d = _match(lam, ref.lam)
    assert np.all(d <= 1e-10 * np.maximum(1.0, np.abs(ref.lam[j])))
    X = X.cpu().numpy()
    for a, b in zip(i, j):
        assert abs(np.vdot(ref.X[:, b], X[:, a])) >= 1 - 1e-10
    # one pass of Algorithm 1 with t close to s: residuals near 1e-9 on both sides,
    # equal to a few digits (the library forms them from (A U) y, the oracle from A (U y))
    r_ref = ref.r[j]
    assert np.all(res[i] <= 1e-8) and np.all(np.abs(res[i] - r_ref) <= 1e-2 * r_ref + 1e-13)
    _, _, dd = _match(lam, p.d[p.inside_mask])
    assert np.all(dd <= 1e-8)


def test_cirr_rejects_a_block_wider_than_m():
    p = pg.make_pencil(200, m=16, inside=6, inside_radius=0.8, outside_r=(2.0, 9.0), seed=62)
    A, B, Yd = to_dev(p.A, p.B, p.V[:, :5])
    with fm.Plan(p.n, 16, p.center, p.radius, p.nodes) as plan:
        with pytest.raises(fm.FeastError) as e:
            plan.cirr(A, B, Yd, 4)          # 5 x 4 = 20 > m = 16
        assert e.value.code == fm.FEAST_EINVAL


def test_cirr_full_size_metric_pencil():
    """Workload 2 (n = 4000, N = 32, s = 100) with h = 32, g = 5 (t = 160 = m):
    one pass of Algorithm 1 finds the 100 eigenvalues; its accuracy is set by
    the quadrature and t (no outer iteration): eigenvalues within 1e-8 of the
    planted ones, residuals up to a few 1e-6 (Algorithm 5 reaches 1e-10)."""
    p = pg.workload(2)
    A, B, Yd = to_dev(p.A, p.B, p.V[:, :32])
    with fm.Plan(p.n, 160, p.center, p.radius, p.nodes, prec=fm.MIXED) as plan:
        lam, X, res, info = plan.cirr(A, B, Yd, 5)
    assert info["t"] == 160 and len(lam) == 100
    _, _, d = _match(lam, p.d[p.inside_mask])
    assert np.all(d <= 1e-8 * np.abs(p.d[p.inside_mask]).max())
    assert np.all(res < 1e-4)
