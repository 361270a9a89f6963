"""C-ABI tests that need no GPU: exported symbols, argument validation, and
the host-side pieces of Algorithm 5 (quadrature nodes, stopping rules and the
reduced-pencil QZ) against the oracle and brute force."""
import math
import os
import re
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import linear_sum_assignment

import paper_1404_1768_amd as fm
from paper_1404_1768_amd import binding as bd
from oracle import gfeast as o
from conftest import ROOT, load_example31


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "feast.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*(feast_[a-z0-9_]+)\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    names = _header_functions()
    assert len(names) >= 14
    lib = fm.load()
    out = subprocess.run(["nm", "-D", "--defined-only", fm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (feast_\w+)", out))
    for nm in names:
        assert nm in exported, nm
        assert hasattr(lib, nm)
    assert set(bd.EXPORTED) == set(names)


def test_version():
    assert fm.load().feast_version() >= 10000


@pytest.mark.parametrize("rule", [fm.TRAPEZOID, fm.GAUSS_LEGENDRE])
@pytest.mark.parametrize("N", [1, 2, 7, 16, 32, 64])
def test_nodes_match_oracle(rule, N):
    z, w = fm.feast_nodes(0.3 - 1.2j, 2.5, N, rule)
    zo, wo = o.contour_nodes(0.3 - 1.2j, 2.5, N, rule)
    assert np.max(np.abs(z - zo)) < 1e-13
    assert np.max(np.abs(w - wo)) < 1e-13


@pytest.mark.parametrize("bad", [dict(radius=0.0), dict(radius=-1.0), dict(nodes=0),
                                 dict(nodes=2000), dict(rule=5), dict(radius=float("nan"))])
def test_invalid_contour_rejected(bad):
    kw = dict(center=0.0, radius=1.0, nodes=16, rule=fm.TRAPEZOID)
    kw.update(bad)
    with pytest.raises(fm.FeastError) as e:
        fm.feast_nodes(**kw)
    assert e.value.code == fm.FEAST_EINVAL


@pytest.mark.parametrize("args", [
    dict(n=0, m=1), dict(n=10, m=0), dict(n=10, m=11), dict(n=20000, m=4),
    dict(n=10, m=4, eta=0.0), dict(n=10, m=4, max_iter=0), dict(n=10, m=4, max_iter=65),
    dict(n=10, m=4, prec=7), dict(n=10, m=4, nb=32), dict(n=10, m=4, radius=0.0),
])
def test_plan_create_validates_before_device_work(args):
    kw = dict(center=0.0, radius=1.0, nodes=16)
    kw.update(args)
    n, m = kw.pop("n"), kw.pop("m")
    with pytest.raises(fm.FeastError) as e:
        fm.Plan(n, m, **kw)
    assert e.value.code == fm.FEAST_EINVAL


def test_null_plan_and_pointer_checks():
    lib = fm.load()
    assert lib.feast_filter(None, None, 1, None, 1, None, 1, None, 1) == fm.FEAST_EINVAL
    assert lib.feast_solve(None, None, 1, None, 1, None, 1, None, None, 1, None, None, None, None,
                           None) == fm.FEAST_EINVAL
    assert lib.feast_plan_destroy(None) == fm.FEAST_OK
    assert lib.feast_zgetrf_batched(0, 1, None, 1, 1, None, None, 0, None) == fm.FEAST_EINVAL
    assert lib.feast_zgemm_batched(1, 4, 4, 4, bd.FeastZ(1, 0), None, 4, 0, None, 4, 0,
                                   bd.FeastZ(0, 0), None, 4, 0, 1, None) == fm.FEAST_EINVAL
    # empty product is a no-op
    assert lib.feast_zgemm_batched(0, 0, 4, 4, bd.FeastZ(1, 0), None, 4, 0, None, 4, 0,
                                   bd.FeastZ(0, 0), None, 4, 0, 1, None) == fm.FEAST_OK


@pytest.mark.parametrize("case", ["count0", "m_gt_n", "n_big", "nodes_differ", "bad_radius",
                                  "prec", "max_iter"])
def test_batch_create_validates_before_device_work(case):
    ns, ms = [100, 60], [10, 6]
    centers, radii, nodes = [0.0, 1.0], [1.0, 1.0], 16
    kw = {}
    if case == "count0":
        ns, ms, centers, radii = [], [], [], []
    elif case == "m_gt_n":
        ms = [10, 61]
    elif case == "n_big":
        ns = [100, 20000]
    elif case == "bad_radius":
        radii = [1.0, 0.0]
    elif case == "prec":
        kw["prec"] = 3
    elif case == "max_iter":
        kw["max_iter"] = 0
    if case == "nodes_differ":
        lib = fm.load()
        c = (bd.Contour * 2)(bd.contour(0.0, 1.0, 16), bd.contour(1.0, 1.0, 8))
        h = bd.C.c_void_p()
        rc = lib.feast_batch_create(bd.C.byref(h), 2, (bd.C.c_int64 * 2)(*ns),
                                    (bd.C.c_int64 * 2)(*ms), c, None, None)
        assert rc == fm.FEAST_EINVAL and not h.value
        return
    with pytest.raises(fm.FeastError) as e:
        fm.Batch(ns, ms, centers, radii, nodes, **kw)
    assert e.value.code == fm.FEAST_EINVAL


def test_null_batch_checks():
    lib = fm.load()
    assert lib.feast_batch_destroy(None) == fm.FEAST_OK
    assert lib.feast_batch_invalidate(None) == fm.FEAST_EINVAL
    assert lib.feast_batch_filter(None, None, None, None, None, None, None, None, None, 0) == fm.FEAST_EINVAL
    assert lib.feast_batch_solve(None, None, None, None, None, None, None, None, None, None, None,
                                 None, None, None, None, None) == fm.FEAST_EINVAL
    assert lib.feast_batch_last_error(None) == b"null batch"


def test_stop_rule_matches_oracle_on_random_sequences():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        k = int(rng.integers(1, 8))
        mx = int(rng.integers(1, 8))
        c_k, c_p = int(rng.integers(0, 3)), int(rng.integers(0, 3))
        e_k = math.inf if c_k == 0 else float(10.0 ** rng.uniform(-14, -2))
        e_p = float(rng.choice([0.0, math.inf, 10.0 ** rng.uniform(-14, -2), e_k]))
        eps = float(10.0 ** rng.uniform(-12, -8))
        assert fm.feast_stop_rule(k, c_k, e_k, c_p, e_p, eps, mx) == \
            o.stop_rule(k, c_k, e_k, c_p, e_p, eps, mx)


def _match(lam, ref):
    C = np.abs(lam[:, None] - ref[None, :])
    ri, ci = linear_sum_assignment(C)
    return C[ri, ci].max()


@pytest.mark.parametrize("t", [1, 2, 3, 9, 40, 120])
def test_reduced_eig_against_brute_force(t):
    rng = np.random.default_rng(t)
    A = rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))
    B = rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))
    al, be, Y = fm.feast_reduced_eig(A, B)
    ref = sla.eigvals(A, B)
    lam = al / be
    assert _match(lam, ref) < 1e-10 * max(1.0, np.abs(ref).max())
    for i in range(t):
        assert abs(np.linalg.norm(Y[:, i]) - 1) < 1e-12
        r = np.linalg.norm(be[i] * A @ Y[:, i] - al[i] * B @ Y[:, i])
        assert r <= 1e-13 * (abs(be[i]) * np.linalg.norm(A) + abs(al[i]) * np.linalg.norm(B))


@pytest.mark.parametrize("t", [1, 2, 3, 5, 17, 64, 97, 160, 255, 256])
def test_reduced_eig_triangular_B_standard_form(t):
    # The method's projected B is upper triangular (R_2 of the QR of B U_1):
    # the solver then works on B^{-1} A; eigenvalues against brute force and
    # every eigenvector's residual with the original pair.
    rng = np.random.default_rng(100 + t)
    A = (rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))) / np.sqrt(t)
    B = np.triu(0.05 * (rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))))
    B[np.diag_indices(t)] = 1.0 + 0.2 * rng.normal(size=t)
    al, be, Y = fm.feast_reduced_eig(A, B)
    assert np.all(be == 1.0)
    ref = sla.eigvals(A, B)
    assert _match(al, ref) < 1e-11 * max(1.0, np.abs(ref).max())
    nA, nB = np.linalg.norm(A), np.linalg.norm(B)
    for i in range(t):
        assert abs(np.linalg.norm(Y[:, i]) - 1) < 1e-12
        r = np.linalg.norm(A @ Y[:, i] - al[i] * B @ Y[:, i])
        assert r <= 1e-12 * (nA + abs(al[i]) * nB), (i, r)


def test_reduced_eig_triangular_B_clusters_and_ritz_like_spectrum():
    # A projected pencil as the method produces it: 40 eigenvalues of a known
    # block in a disk (two pairs 1e-9 apart), 20 spurious ones elsewhere, a
    # rounding-level lower triangle in B (the GEMM-computed U_2^* B U_1).
    rng = np.random.default_rng(7)
    t = 60
    d = 0.8 * np.sqrt(rng.uniform(size=t)) * np.exp(2j * np.pi * rng.uniform(size=t))
    d[40:] = 3.0 * d[40:] + 2.0
    d[1] = d[0] + 1e-9
    d[3] = d[2] + 1e-9j
    S = np.eye(t) + 0.1 * (rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))) / np.sqrt(t)
    R = np.triu(np.eye(t) + 0.05 * (rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))))
    A = R @ S @ np.diag(d) @ np.linalg.inv(S)
    B = R + 1e-17 * np.tril(rng.normal(size=(t, t)), -1)
    al, be, Y = fm.feast_reduced_eig(A, B)
    lam = al / be
    assert _match(lam, d) < 1e-9
    nA, nB = np.linalg.norm(A), np.linalg.norm(B)
    for i in range(t):
        r = np.linalg.norm(A @ Y[:, i] - lam[i] * B @ Y[:, i])
        assert r <= 1e-12 * (nA + abs(lam[i]) * nB), (i, r)


def test_reduced_eig_tiny_couplings_keep_full_accuracy():
    # A nearly decoupled block: entries 1e-11 below a 4.5e-2 subdiagonal must
    # still be reduced (their sum of squares is below the rounding of the
    # column's), or the Hessenberg form is lost at the 1e-11 level.
    M = np.array([[0.49, 0.045, 1e-11], [0.045, 0.2, 2e-9], [1e-11, 2e-9, 2.0]], complex)
    al, be, Y = fm.feast_reduced_eig(M, np.eye(3, dtype=complex))
    assert _match(al / be, np.linalg.eigvals(M)) < 1e-15
    for i in range(3):
        assert np.linalg.norm(M @ Y[:, i] - al[i] / be[i] * Y[:, i]) < 1e-15


def test_reduced_eig_infinite_eigenvalues():
    # a rank-deficient Bt gives beta = 0 for as many eigenvalues as its rank defect
    rng = np.random.default_rng(2)
    t = 14
    A = rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))
    B = rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))
    U, s, Vh = np.linalg.svd(B)
    s[-3:] = 0
    B = (U * s) @ Vh
    al, be, Y = fm.feast_reduced_eig(A, B)
    inf = np.abs(be) < 1e-12 * np.abs(al)
    assert np.count_nonzero(inf) == 3
    ref = sla.eigvals(A, B)
    assert _match(al[~inf] / be[~inf], ref[np.isfinite(ref)]) < 1e-9


def test_reduced_eig_example31_projection():
    # Section 3: the oblique reduced pencil of Example 3.1 has eigenvalues 0.2, 0.5
    A, B, eig = load_example31()
    z, w = o.contour_nodes(0.0, 1.0, 32)
    V = np.array([[0.3, -1.1], [0.7, 0.2], [-0.4, 0.9], [1.3, 0.5]], dtype=np.complex128)
    U1, _ = o.orth(o.apply_filter(o.ShiftedSolver(A, B, z), w, V))
    U2, _ = o.orth(B @ U1)
    At, Bt = o.project(A, B, U1, U2)
    al, be, Y = fm.feast_reduced_eig(At, Bt)
    assert np.allclose(np.sort((al / be).real), [0.2, 0.5], atol=1e-9)


def test_reduced_eig_triangular_and_diagonal_inputs():
    t = 6
    D = np.diag(np.arange(1, t + 1) * (1 + 0.5j))
    al, be, Y = fm.feast_reduced_eig(D, np.eye(t))
    assert np.allclose(np.sort_complex(al / be), np.sort_complex(np.diag(D)))
    T = np.triu(np.ones((t, t))) + np.diag(np.arange(t))
    al, be, Y = fm.feast_reduced_eig(T + 0j, np.eye(t) + 0j)
    assert np.allclose(np.sort((al / be).real), np.sort(np.diag(T)))


@pytest.mark.parametrize("sa,sb", [(1e30, 1e30), (1e-30, 1e-30), (1e30, 1e-30), (1e-30, 1e30)])
@pytest.mark.parametrize("tri", [False, True])
def test_reduced_eig_badly_scaled_pencils(sa, sb, tri):
    # The host solver's complex arithmetic does not scale its divisions (it is
    # built with limited-range complex arithmetic for speed): this pins that
    # pencils scaled by 1e+-30 -- eigenvalues scaled by up to 1e+-60 -- keep
    # full relative accuracy, in the standard-form (triangular B) and QZ paths.
    rng = np.random.default_rng(31)
    t = 48
    A = (rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))) / np.sqrt(t)
    if tri:
        B = np.triu(0.05 * (rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))))
        B[np.diag_indices(t)] = 1.0 + 0.2 * rng.normal(size=t)
    else:
        B = rng.normal(size=(t, t)) + 1j * rng.normal(size=(t, t))
    ref = sla.eigvals(A, B)
    al, be, Y = fm.feast_reduced_eig(sa * A, sb * B)
    lam = al / be * (sb / sa)
    assert np.all(np.isfinite(lam))
    assert _match(lam, ref) < 1e-10 * max(1.0, np.abs(ref).max())
    for i in range(t):
        assert abs(np.linalg.norm(Y[:, i]) - 1) < 1e-12
        # beta sa A y = alpha sb B y  <=>  (beta / sb) A y = (alpha / sa) B y
        r = np.linalg.norm(be[i] / sb * (A @ Y[:, i]) - al[i] / sa * (B @ Y[:, i]))
        assert r <= 1e-12 * (abs(be[i] / sb) * np.linalg.norm(A) + abs(al[i] / sa) * np.linalg.norm(B))


def test_binding_structs_match_the_header(tmp_path):
    # The ctypes mirrors of the header's structs must have the C layout:
    # compile a probe against include/feast.h and compare sizes and offsets.
    import ctypes
    import shutil
    import subprocess
    from paper_1404_1768_amd import binding as b
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "probe.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "feast.h"\n'
        'int main(void) {\n'
        '  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(feast_contour), sizeof(feast_opts),\n'
        '         sizeof(feast_info), sizeof(feast_search_info), sizeof(feast_cirr_info),\n'
        '         sizeof(feast_batch_info), offsetof(feast_info, hbm));\n'
        '  return 0;\n}\n')
    exe = tmp_path / "probe"
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [ctypes.sizeof(t) for t in (b.Contour, b.Opts, b.Info, b.SearchInfo, b.CirrInfo,
                                       b.BatchInfo)] + [b.Info.hbm.offset]
    assert got == want


def test_noalloc_solve_checks_sizes_before_device_work():
    # Argument and scratch-size checks of feast_zgetrs_batched_noalloc come
    # before any device call: placeholder pointers are never dereferenced.
    lib = fm.load()
    import ctypes
    fake = ctypes.c_void_p(0x1000)
    big = lib.feast_zgetrs_batched_noalloc(16384, 1000, 1, fake, 16384, 16384 * 16384, fake, fake,
                                           1000, 16384 * 1000, 0, None)
    assert big == fm.FEAST_ESCRATCH
    assert lib.feast_zgetrs_batched_noalloc(0, 4, 1, fake, 1, 1, fake, fake, 4, 4, 0, None) == \
        fm.FEAST_EINVAL
    assert lib.feast_zgetrs_batched_noalloc(8, 4, 1, fake, 8, 64, fake, fake, 4, 32, 1, None) == \
        fm.FEAST_EINVAL
    assert lib.feast_zgetrs_batched_noalloc(8, 4, 1, None, 8, 64, fake, fake, 4, 32, 0, None) == \
        fm.FEAST_EINVAL
