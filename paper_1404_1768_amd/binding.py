"""ctypes binding of ``libfeast_mi355x.so`` (the C ABI declared in ``include/feast.h``).

Argument marshalling only: every step of the method runs in the library.
PyTorch supplies device memory and the stream.  Tensors must be complex128,
two-dimensional and row-major with unit column stride (``ld = t.stride(0)``).
The library must have been built (``python -m paper_1404_1768_amd.build``);
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfeast_mi355x.so")

FEAST_OK = 0
FEAST_SINGULAR = 1
FEAST_REFINE_STAGNATED = 2
FEAST_EINVAL = -1
FEAST_EDEVICE = -2
FEAST_ENOMEM = -3
FEAST_ENUMERIC = -4
FEAST_ESCRATCH = -5

TRAPEZOID = 0
GAUSS_LEGENDRE = 1
FP64 = 0
MIXED = 1
MAX_HISTORY = 64

EXPORTED = [
    "feast_opts_default", "feast_nodes", "feast_plan_create", "feast_plan_destroy",
    "feast_plan_invalidate", "feast_filter", "feast_project", "feast_solve", "feast_last_error",
    "feast_reduced_eig", "feast_stop_rule", "feast_zgetrf_batched", "feast_zgetrs_batched",
    "feast_zgemm_batched", "feast_version", "feast_left_eigvecs", "feast_eig_grad",
    "feast_batch_create", "feast_batch_destroy", "feast_batch_invalidate",
    "feast_batch_last_error", "feast_batch_filter", "feast_batch_solve",
    "feast_search", "feast_plan_set_m", "feast_solve_from", "feast_enclosing_circle",
    "feast_region_select", "feast_cirr", "feast_zgetrs_batched_noalloc", "feast_solve_csr",
    "feast_csr_order",
]


class FeastZ(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Contour(C.Structure):
    _fields_ = [("center", FeastZ), ("radius", C.c_double), ("nodes", C.c_int32),
                ("rule", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("eta", C.c_double), ("max_iter", C.c_int32),
                ("prec", C.c_int32), ("refine_tol", C.c_double), ("max_sweeps", C.c_int32),
                ("nb", C.c_int32), ("profile", C.c_int32), ("lookahead", C.c_int32),
                ("update_tile", C.c_int32), ("batch_update", C.c_int32),
                ("ahead_cus", C.c_int32), ("ahead_rows", C.c_int32)]


K_CLASSES = ["shift", "weighted_sum", "gather_rows", "z_to_c", "c_to_z", "fingerprint"]


class KProf(C.Structure):
    _fields_ = [("launches", C.c_int32), ("ms", C.c_double), ("bytes", C.c_double)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("filters", C.c_int32),
                ("count", C.c_int32 * MAX_HISTORY), ("err", C.c_double * MAX_HISTORY),
                ("sweeps", C.c_int32 * MAX_HISTORY),
                ("t_factor_ms", C.c_double), ("t_filter_ms", C.c_double),
                ("t_project_ms", C.c_double), ("t_host_eig_ms", C.c_double),
                ("t_ritz_ms", C.c_double), ("t_total_ms", C.c_double),
                ("lu_gemm_launches", C.c_int32), ("lu_gemm_ms", C.c_double),
                ("lu_gemm_flops", C.c_double), ("hbm", KProf * len(K_CLASSES)),
                ("contraction", C.c_double * MAX_HISTORY),
                ("band_kl", C.c_int32), ("band_ku", C.c_int32), ("fp64_fallback", C.c_int32)]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class SearchInfo(C.Structure):
    _fields_ = [("t", C.c_int64), ("s0", C.c_int64), ("used", C.c_int64),
                ("rounds", C.c_int32), ("filters", C.c_int32), ("ms", C.c_double)]


class CirrInfo(C.Structure):
    _fields_ = [("t", C.c_int64), ("ms", C.c_double)]


class BatchInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("filters", C.c_int32), ("graph_launches", C.c_int32),
                ("t_factor_ms", C.c_double), ("t_filter_ms", C.c_double),
                ("t_project_ms", C.c_double), ("t_host_eig_ms", C.c_double),
                ("t_total_ms", C.c_double)]


class FeastError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("feast error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            "%s is missing: build it with `python -m paper_1404_1768_amd.build`" % path)
    lib = C.CDLL(path)
    P = C.c_void_p
    i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
    pz = C.POINTER(FeastZ)
    lib.feast_opts_default.argtypes = [C.POINTER(Opts)]
    lib.feast_opts_default.restype = None
    lib.feast_nodes.argtypes = [C.POINTER(Contour), pz, pz]
    lib.feast_plan_create.argtypes = [C.POINTER(P), i64, i64, C.POINTER(Contour), C.POINTER(Opts), P]
    lib.feast_plan_destroy.argtypes = [P]
    lib.feast_plan_invalidate.argtypes = [P]
    lib.feast_filter.argtypes = [P, P, i64, P, i64, P, i64, P, i64]
    lib.feast_project.argtypes = [P, P, i64, P, i64, P, i64, P, i64, P, i64, pz, pz]
    lib.feast_solve.argtypes = [P, P, i64, P, i64, P, i64, pz, P, i64, C.POINTER(dbl),
                                C.POINTER(i32), C.POINTER(dbl), C.POINTER(i32), C.POINTER(Info)]
    lib.feast_solve_from.argtypes = list(lib.feast_solve.argtypes)
    lib.feast_solve_csr.argtypes = [P, C.POINTER(Csr), C.POINTER(Csr), P, i64, pz, P, i64,
                                    C.POINTER(dbl), C.POINTER(i32), C.POINTER(dbl), C.POINTER(i32),
                                    C.POINTER(Info)]
    lib.feast_csr_order.argtypes = [i64, P, P, P, C.POINTER(i64), C.POINTER(i64)]
    lib.feast_search.argtypes = [P, P, i64, P, i64, P, i64, i64, i32, dbl, dbl, P, i64,
                                 C.POINTER(SearchInfo)]
    lib.feast_plan_set_m.argtypes = [P, i64]
    lib.feast_cirr.argtypes = [P, P, i64, P, i64, P, i64, i32, i32, pz, P, i64, C.POINTER(dbl),
                               C.POINTER(i32), C.POINTER(CirrInfo)]
    lib.feast_enclosing_circle.argtypes = [i32, pz, dbl, pz, C.POINTER(dbl)]
    lib.feast_region_select.argtypes = [i32, pz, i64, pz, C.POINTER(i32)]
    lib.feast_last_error.argtypes = [P]
    lib.feast_last_error.restype = C.c_char_p
    lib.feast_reduced_eig.argtypes = [i64, pz, i64, pz, i64, pz, pz, pz, i64]
    lib.feast_stop_rule.argtypes = [i32, i32, dbl, i32, dbl, dbl, i32]
    lib.feast_zgetrf_batched.argtypes = [i64, i32, P, i64, i64, P, P, i32, P]
    lib.feast_zgetrs_batched.argtypes = [i64, i64, i32, P, i64, i64, P, P, i64, i64, i32, P]
    lib.feast_zgetrs_batched_noalloc.argtypes = list(lib.feast_zgetrs_batched.argtypes)
    lib.feast_zgemm_batched.argtypes = [i32, i64, i64, i64, FeastZ, P, i64, i64, P, i64, i64,
                                        FeastZ, P, i64, i64, i32, P]
    lib.feast_left_eigvecs.argtypes = [P, P, i64, P, i64, P, i64, i64, i32, P, i64]
    lib.feast_eig_grad.argtypes = [P, P, i64, P, i64, i64, pz, pz, P, i64, P, i64]
    pi64, pp = C.POINTER(i64), C.POINTER(P)
    lib.feast_batch_create.argtypes = [C.POINTER(P), i32, pi64, pi64, C.POINTER(Contour),
                                       C.POINTER(Opts), P]
    lib.feast_batch_destroy.argtypes = [P]
    lib.feast_batch_invalidate.argtypes = [P]
    lib.feast_batch_last_error.argtypes = [P]
    lib.feast_batch_last_error.restype = C.c_char_p
    lib.feast_batch_filter.argtypes = [P, pp, pi64, pp, pi64, pp, pi64, pp, pi64, i32]
    lib.feast_batch_solve.argtypes = [P, pp, pi64, pp, pi64, pp, pi64, pp, pp, pi64, pp,
                                      C.POINTER(i32), C.POINTER(dbl), C.POINTER(i32),
                                      C.POINTER(i32), C.POINTER(BatchInfo)]
    for name in EXPORTED:
        if name not in ("feast_opts_default", "feast_last_error", "feast_batch_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _zptr(a: np.ndarray):
    assert a.dtype == np.complex128 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(FeastZ))


def _dev(t, rows=None, cols=None, name="tensor"):
    """(pointer, ld) of a device complex128 row-major matrix."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.complex128 or t.dim() != 2 or not t.is_cuda:
        raise ValueError("%s must be a 2-D complex128 CUDA tensor" % name)
    if t.stride(1) != 1 or (t.shape[0] > 1 and t.stride(0) < t.shape[1]):
        raise ValueError("%s must be row-major with unit column stride" % name)
    if rows is not None and t.shape[0] != rows:
        raise ValueError("%s has %d rows, expected %d" % (name, t.shape[0], rows))
    if cols is not None and t.shape[1] != cols:
        raise ValueError("%s has %d columns, expected %d" % (name, t.shape[1], cols))
    return C.c_void_p(t.data_ptr()), max(t.stride(0), t.shape[1])


def _csr(M, n, name):
    """feast_csr of an n x n CSR matrix given as (rowptr, col, val) device
    tensors: int32 (n + 1), int32 (nnz), complex128 (nnz)."""
    import torch
    rp, ci, va = M
    for t, dt, what in ((rp, torch.int32, "rowptr"), (ci, torch.int32, "col"),
                        (va, torch.complex128, "val")):
        if not isinstance(t, torch.Tensor) or t.dtype != dt or t.dim() != 1 or not t.is_cuda \
                or not t.is_contiguous():
            raise ValueError("%s.%s must be a contiguous 1-D %s CUDA tensor" % (name, what, dt))
    if rp.numel() != n + 1 or ci.numel() != va.numel():
        raise ValueError("%s: rowptr needs n + 1 entries and col, val the same count" % name)
    return Csr(n, ci.numel(), rp.data_ptr(), ci.data_ptr(), va.data_ptr())


def csr_order(rowptr: np.ndarray, col: np.ndarray):
    """Host: the ordering feast_solve_csr uses for a CSR pattern (reverse
    Cuthill-McKee of the symmetrised pattern, or the natural order where that
    is at least as narrow): (perm with perm[new] = old, kl, ku in that order)."""
    lib = load()
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    n = rp.size - 1
    perm = np.zeros(n, dtype=np.int32)
    kl, ku = C.c_int64(), C.c_int64()
    rc = lib.feast_csr_order(n, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                           perm.ctypes.data_as(C.c_void_p), C.byref(kl), C.byref(ku))
    if rc != FEAST_OK:
        raise FeastError(rc, "feast_csr_order: malformed pattern")
    return perm, int(kl.value), int(ku.value)


def _stream(stream):
    import torch
    if stream is None:
        if not torch.cuda.is_available():
            return C.c_void_p(None)
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def contour(center: complex, radius: float, nodes: int, rule: int = TRAPEZOID) -> Contour:
    c = complex(center)
    return Contour(FeastZ(c.real, c.imag), float(radius), int(nodes), int(rule))


def default_opts() -> Opts:
    o = Opts()
    load().feast_opts_default(C.byref(o))
    return o


# ---------------------------------------------------------------------------
# host-only entry points
# ---------------------------------------------------------------------------

def feast_nodes(center: complex, radius: float, nodes: int, rule: int = TRAPEZOID):
    lib = load()
    z = np.zeros(nodes, dtype=np.complex128)
    w = np.zeros(nodes, dtype=np.complex128)
    c = contour(center, radius, nodes, rule)
    rc = lib.feast_nodes(C.byref(c), _zptr(z), _zptr(w))
    if rc != FEAST_OK:
        raise FeastError(rc, "invalid contour")
    return z, w


def feast_reduced_eig(At: np.ndarray, Bt: np.ndarray):
    lib = load()
    At = np.ascontiguousarray(At, dtype=np.complex128)
    Bt = np.ascontiguousarray(Bt, dtype=np.complex128)
    t = At.shape[0]
    if At.shape != (t, t) or Bt.shape != (t, t):
        raise ValueError("square matrices of equal size expected")
    al = np.zeros(t, dtype=np.complex128)
    be = np.zeros(t, dtype=np.complex128)
    Y = np.zeros((t, t), dtype=np.complex128)
    rc = lib.feast_reduced_eig(t, _zptr(At), t, _zptr(Bt), t, _zptr(al), _zptr(be), _zptr(Y), t)
    if rc != FEAST_OK:
        raise FeastError(rc, "reduced eigensolver failed")
    return al, be, Y


def feast_stop_rule(k, c_k, e_k, c_prev, e_prev, eps, max_iter) -> int:
    return load().feast_stop_rule(k, c_k, float(e_k), c_prev, float(e_prev), float(eps), max_iter)


def enclosing_circle(vertices, margin: float = 0.1):
    """(center, radius) of the smallest circle enclosing the polygon's
    vertices, radius enlarged by (1 + margin)."""
    v = np.ascontiguousarray(vertices, dtype=np.complex128).ravel()
    c = FeastZ()
    r = C.c_double()
    rc = load().feast_enclosing_circle(v.size, _zptr(v), float(margin), C.byref(c), C.byref(r))
    if rc != FEAST_OK:
        raise FeastError(rc, "feast_enclosing_circle: bad vertices or margin")
    return complex(c.re, c.im), r.value


def region_inside(vertices, lam) -> np.ndarray:
    """Boolean mask of the points lam inside the polygon (even-odd rule)."""
    v = np.ascontiguousarray(vertices, dtype=np.complex128).ravel()
    z = np.ascontiguousarray(lam, dtype=np.complex128).ravel()
    out = np.zeros(z.size, dtype=np.int32)
    rc = load().feast_region_select(v.size, _zptr(v), z.size, _zptr(z),
                                    out.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc != FEAST_OK:
        raise FeastError(rc, "feast_region_select: bad arguments")
    return out.astype(bool)


def solve_region(A, B, V, vertices, nodes: int = 32, margin: float = 0.1, **plan_kw):
    """Eigenpairs inside an irregular closed curve (a polygon): Algorithm 5 on
    the enclosing circle, then the pairs inside the polygon (Section 4.3).
    Returns (SolveResult restricted to the region, (center, radius))."""
    center, radius = enclosing_circle(vertices, margin)
    n, m = int(A.shape[0]), int(V.shape[1])
    with Plan(n, m, center, radius, nodes, **plan_kw) as plan:
        r = plan.solve(A, B, V)
    keep = region_inside(vertices, r.lam)
    idx = np.flatnonzero(keep)
    r = dataclasses.replace(r, lam=r.lam[idx], X=r.X[:, idx], res=r.res[idx])
    return r, (center, radius)


# ---------------------------------------------------------------------------
# plan
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SolveResult:
    lam: np.ndarray        # selected eigenvalues
    X: object              # torch tensor n x s (device)
    res: np.ndarray        # residuals r_i of eq. (5-1)
    err: float
    flag: int
    iters: int
    filters: int
    count: list
    errs: list
    sweeps: list
    times: dict
    status: int
    lu_gemm: dict
    hbm: dict = dataclasses.field(default_factory=dict)
    contraction: list = dataclasses.field(default_factory=list)
    band: tuple = None     # feast_solve_csr: (kl, ku) of the reordered pencil
    fp64_fallback: int = 0  # mixed form: filter after which the solve switched to FP64 (0: none)


class Plan:
    """A FEAST plan: contour, options, device workspace and cached LU factors."""

    def __init__(self, n: int, m: int, center: complex, radius: float, nodes: int,
                 rule: int = TRAPEZOID, eps: float = 1e-10, eta: float = 1e-3,
                 max_iter: int = 20, prec: int = FP64, refine_tol: Optional[float] = None,
                 max_sweeps: int = 6, nb: int = 0, profile: bool = False,
                 lookahead: Optional[bool] = None, update_tile: Optional[int] = None,
                 ahead_cus: Optional[int] = None, ahead_rows: Optional[int] = None,
                 stream=None):
        self.lib = load()
        self.n, self.m = int(n), int(m)
        self.contour = contour(center, radius, nodes, rule)
        self.opts = default_opts()
        self.opts.eps, self.opts.eta, self.opts.max_iter = float(eps), float(eta), int(max_iter)
        self.opts.prec, self.opts.max_sweeps, self.opts.nb = int(prec), int(max_sweeps), int(nb)
        self.opts.profile = 1 if profile else 0
        if lookahead is not None:
            self.opts.lookahead = 1 if lookahead else 0
        if update_tile is not None:
            self.opts.update_tile = int(update_tile)
        if ahead_cus is not None:
            self.opts.ahead_cus = int(ahead_cus)
        if ahead_rows is not None:
            self.opts.ahead_rows = int(ahead_rows)
        if refine_tol is not None:
            self.opts.refine_tol = float(refine_tol)
        self._stream_obj = stream
        self._h = C.c_void_p()
        rc = self.lib.feast_plan_create(C.byref(self._h), self.n, self.m, C.byref(self.contour),
                                        C.byref(self.opts), _stream(stream))
        if rc != FEAST_OK:
            raise FeastError(rc, "feast_plan_create failed")

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if self._h:
            self.lib.feast_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return self.lib.feast_last_error(self._h).decode()

    def _check(self, rc, what, ok=(FEAST_OK,)):
        if rc not in ok:
            raise FeastError(rc, "%s: %s" % (what, self.last_error()))
        return rc

    def invalidate(self):
        self._check(self.lib.feast_plan_invalidate(self._h), "feast_plan_invalidate")

    # -- the three calls ---------------------------------------------------
    def filter(self, A, B, V, U=None, allow=(FEAST_OK,)):
        import torch
        n, m = self.n, self.m
        pa, lda = _dev(A, n, n, "A")
        pb, ldb = _dev(B, n, n, "B")
        pv, ldv = _dev(V, n, m, "V")
        if U is None:
            U = torch.empty((n, m), dtype=torch.complex128, device=V.device)
        pu, ldu = _dev(U, n, m, "U")
        rc = self.lib.feast_filter(self._h, pa, lda, pb, ldb, pv, ldv, pu, ldu)
        self.status = self._check(rc, "feast_filter", ok=(FEAST_OK,) + tuple(allow))
        return U

    def project(self, A, B, U):
        import torch
        n, m = self.n, self.m
        pa, lda = _dev(A, n, n, "A")
        pb, ldb = _dev(B, n, n, "B")
        pu, ldu = _dev(U, n, m, "U")
        AU1 = torch.empty((n, m), dtype=torch.complex128, device=U.device)
        BU1 = torch.empty((n, m), dtype=torch.complex128, device=U.device)
        At = np.zeros((m, m), dtype=np.complex128)
        Bt = np.zeros((m, m), dtype=np.complex128)
        rc = self.lib.feast_project(self._h, pa, lda, pb, ldb, pu, ldu,
                                    C.c_void_p(AU1.data_ptr()), m, C.c_void_p(BU1.data_ptr()), m,
                                    _zptr(At), _zptr(Bt))
        self._check(rc, "feast_project")
        return U, AU1, BU1, At, Bt

    def solve(self, A, B, V, allow=(FEAST_REFINE_STAGNATED,)) -> SolveResult:
        return self._solve(self.lib.feast_solve, "feast_solve", A, B, V, allow)

    def solve_from(self, A, B, U1, allow=(FEAST_REFINE_STAGNATED,)) -> SolveResult:
        """Algorithm 5 after its Search call, from Search's orthonormal basis U1 (n x m)."""
        return self._solve(self.lib.feast_solve_from, "feast_solve_from", A, B, U1, allow)

    def _solve(self, fn, what, A, B, V, allow) -> SolveResult:
        import torch
        n, m = self.n, self.m
        pa, lda = _dev(A, n, n, "A")
        pb, ldb = _dev(B, n, n, "B")
        pv, ldv = _dev(V, n, m, "V")
        X = torch.empty((n, m), dtype=torch.complex128, device=V.device)
        lam = np.zeros(m, dtype=np.complex128)
        res = np.zeros(m, dtype=np.float64)
        s = C.c_int32()
        err = C.c_double()
        flag = C.c_int32()
        info = Info()
        rc = fn(self._h, pa, lda, pb, ldb, pv, ldv, _zptr(lam), C.c_void_p(X.data_ptr()), m,
                res.ctypes.data_as(C.POINTER(C.c_double)), C.byref(s), C.byref(err),
                C.byref(flag), C.byref(info))
        self._check(rc, what, ok=(FEAST_OK,) + tuple(allow))
        return self._result(rc, info, lam, res, X, s, err, flag)

    def solve_csr(self, A, B, V, allow=(FEAST_REFINE_STAGNATED,)) -> SolveResult:
        """Algorithm 5 for a sparse pencil: A and B as (rowptr, col, val) device
        tensors (int32, int32, complex128) of n x n CSR matrices; FP64 plans
        only.  The result's `band` is (kl, ku) of the reordered pencil."""
        import torch
        n, m = self.n, self.m
        ca, cb = _csr(A, n, "A"), _csr(B, n, "B")
        pv, ldv = _dev(V, n, m, "V")
        X = torch.empty((n, m), dtype=torch.complex128, device=V.device)
        lam = np.zeros(m, dtype=np.complex128)
        res = np.zeros(m, dtype=np.float64)
        s = C.c_int32()
        err = C.c_double()
        flag = C.c_int32()
        info = Info()
        rc = self.lib.feast_solve_csr(self._h, C.byref(ca), C.byref(cb), pv, ldv, _zptr(lam),
                                      C.c_void_p(X.data_ptr()), m,
                                      res.ctypes.data_as(C.POINTER(C.c_double)), C.byref(s),
                                      C.byref(err), C.byref(flag), C.byref(info))
        self._check(rc, "feast_solve_csr", ok=(FEAST_OK,) + tuple(allow))
        out = self._result(rc, info, lam, res, X, s, err, flag)
        out.band = (int(info.band_kl), int(info.band_ku))
        return out

    def _result(self, rc, info, lam, res, X, s, err, flag) -> SolveResult:
        k = s.value
        it = info.iters
        return SolveResult(
            lam=lam[:k].copy(), X=X[:, :k], res=res[:k].copy(), err=err.value, flag=flag.value,
            iters=it, filters=info.filters, count=list(info.count[:it]), errs=list(info.err[:it]),
            sweeps=list(info.sweeps[:info.filters]),
            times={"factor": info.t_factor_ms, "filter": info.t_filter_ms,
                   "project": info.t_project_ms, "host_eig": info.t_host_eig_ms,
                   "ritz": info.t_ritz_ms, "total": info.t_total_ms},
            status=rc, lu_gemm={"launches": info.lu_gemm_launches, "ms": info.lu_gemm_ms,
                                "flops": info.lu_gemm_flops},
            hbm={name: {"launches": info.hbm[i].launches, "ms": info.hbm[i].ms,
                        "bytes": info.hbm[i].bytes}
                 for i, name in enumerate(K_CLASSES) if info.hbm[i].launches > 0},
            contraction=list(info.contraction[:info.filters]), fp64_fallback=int(info.fp64_fallback))

    # -- Search (Algorithm 4) ----------------------------------------------
    def search(self, A, B, Ypool, p: int, alpha: float = 1.5, tau: float = 1e-3):
        """Algorithm 4 with the random columns of Ypool (n x q, N(0,1) entries,
        complex dtype): returns (U1 of shape n x t, info dict with t, s0, used,
        rounds, filters, ms)."""
        import torch
        n, m = self.n, self.m
        pa, lda = _dev(A, n, n, "A")
        pb, ldb = _dev(B, n, n, "B")
        q = int(Ypool.shape[1])
        py, ldy = _dev(Ypool, n, q, "Ypool")
        U1 = torch.empty((n, m), dtype=torch.complex128, device=Ypool.device)
        info = SearchInfo()
        rc = self.lib.feast_search(self._h, pa, lda, pb, ldb, py, ldy, q, int(p), float(alpha),
                                   float(tau), C.c_void_p(U1.data_ptr()), m, C.byref(info))
        self._check(rc, "feast_search")
        t = int(info.t)
        return U1[:, :t], {"t": t, "s0": int(info.s0), "used": int(info.used),
                           "rounds": int(info.rounds), "filters": int(info.filters),
                           "ms": float(info.ms)}

    # -- Block_CIRR (Algorithm 1) -------------------------------------------
    def cirr(self, A, B, Y, g: int):
        """Algorithm 1 with the random block Y (n x h) and g moments (h g <= m):
        returns (lam, X (n x s), res, info dict with t and ms)."""
        import torch
        n, m = self.n, self.m
        pa, lda = _dev(A, n, n, "A")
        pb, ldb = _dev(B, n, n, "B")
        h = int(Y.shape[1])
        py, ldy = _dev(Y, n, h, "Y")
        X = torch.empty((n, m), dtype=torch.complex128, device=Y.device)
        lam = np.zeros(m, dtype=np.complex128)
        res = np.zeros(m, dtype=np.float64)
        s = C.c_int32()
        info = CirrInfo()
        rc = self.lib.feast_cirr(self._h, pa, lda, pb, ldb, py, ldy, h, int(g), _zptr(lam),
                                 C.c_void_p(X.data_ptr()), m,
                                 res.ctypes.data_as(C.POINTER(C.c_double)), C.byref(s),
                                 C.byref(info))
        self._check(rc, "feast_cirr")
        k = s.value
        return lam[:k].copy(), X[:, :k], res[:k].copy(), {"t": int(info.t), "ms": float(info.ms)}

    def set_m(self, m: int):
        """New subspace size, keeping the cached factors."""
        self._check(self.lib.feast_plan_set_m(self._h, int(m)), "feast_plan_set_m")
        self.m = int(m)

    # -- adjoint form ------------------------------------------------------
    def left_eigvecs(self, A, B, X, sweeps: int = 3):
        """Left eigenvectors Y (n x s) with Y^* B X = I from the adjoint filter."""
        import torch
        n = self.n
        pa, lda = _dev(A, n, n, "A")
        pb, ldb = _dev(B, n, n, "B")
        X = X.contiguous()
        s = X.shape[1]
        px, ldx = _dev(X, n, s, "X")
        Y = torch.empty((n, s), dtype=torch.complex128, device=X.device)
        rc = self.lib.feast_left_eigvecs(self._h, pa, lda, pb, ldb, px, ldx, s, int(sweeps),
                                         C.c_void_p(Y.data_ptr()), s)
        self._check(rc, "feast_left_eigvecs")
        return Y

    def eig_grad(self, X, Y, lam, g):
        """(dL/dA, dL/dB) for dL/d conj(lambda_i) = g_i (PyTorch convention)."""
        import torch
        n = self.n
        X = X.contiguous()
        Y = Y.contiguous()
        s = X.shape[1]
        lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128).reshape(s))
        g = np.ascontiguousarray(np.asarray(g, dtype=np.complex128).reshape(s))
        GA = torch.empty((n, n), dtype=torch.complex128, device=X.device)
        GB = torch.empty((n, n), dtype=torch.complex128, device=X.device)
        rc = self.lib.feast_eig_grad(self._h, C.c_void_p(X.data_ptr()), s, C.c_void_p(Y.data_ptr()),
                                     s, s, _zptr(lam), _zptr(g), C.c_void_p(GA.data_ptr()), n,
                                     C.c_void_p(GB.data_ptr()), n)
        self._check(rc, "feast_eig_grad")
        return GA, GB


def _feast_eig_function():
    import torch

    class FeastEig(torch.autograd.Function):
        """Eigenvalues inside the contour as a differentiable function of (A, B).

        Forward: Algorithm 5 (``feast_solve``).  Backward: left eigenvectors from
        the adjoint filter on the forward LU factors (``feast_left_eigvecs``) and
        the rank-s gradient assembly (``feast_eig_grad``)."""

        @staticmethod
        def forward(ctx, A, B, V, plan, sweeps):
            r = plan.solve(A, B, V)
            if r.flag != 1:
                import warnings
                warnings.warn("feast_eig: Algorithm 5 stopped with flag %d (%s), Err = %.3e; the "
                              "eigenvalues and their gradients carry that error" %
                              (r.flag, "no improvement, previous iterate" if r.flag == 0
                               else "iteration cap", r.err), RuntimeWarning, stacklevel=3)
            ctx.plan, ctx.sweeps = plan, sweeps
            ctx.X = r.X.contiguous().clone()
            ctx.lam = r.lam.copy()
            ctx.save_for_backward(A, B)
            ctx.result = r
            return torch.from_numpy(r.lam.copy()).to(A.device)

        @staticmethod
        def backward(ctx, g):
            A, B = ctx.saved_tensors
            Y = ctx.plan.left_eigvecs(A, B, ctx.X, ctx.sweeps)
            GA, GB = ctx.plan.eig_grad(ctx.X, Y, ctx.lam, g.detach().cpu().numpy())
            return GA, GB, None, None, None

    return FeastEig


_FEAST_EIG = None


def feast_eig(A, B, V, plan: "Plan", sweeps: int = 3):
    """Differentiable eigenvalues of (A, B) inside the plan's contour."""
    global _FEAST_EIG
    if _FEAST_EIG is None:
        _FEAST_EIG = _feast_eig_function()
    return _FEAST_EIG.apply(A, B, V, plan, sweeps)


# Module-level functions with the C names.
def feast_filter(plan: Plan, A, B, V, U=None):
    return plan.filter(A, B, V, U)


def feast_project(plan: Plan, A, B, U):
    return plan.project(A, B, U)


def feast_solve(plan: Plan, A, B, V):
    return plan.solve(A, B, V)


# ---------------------------------------------------------------------------
# kernel-level entry points
# ---------------------------------------------------------------------------

def zgemm_batched(A, B, C_, alpha=1.0, beta=0.0, transA=0, stream=None):
    """C_b = alpha op(A_b) B_b + beta C_b on 3-D (batch, rows, cols) complex128 tensors."""
    lib = load()
    for t, nm in ((A, "A"), (B, "B"), (C_, "C")):
        if t.dim() != 3 or t.stride(2) != 1 or t.dtype.is_complex is False:
            raise ValueError("%s must be (batch, rows, cols) row-major" % nm)
    batch = C_.shape[0]
    M, N = C_.shape[1], C_.shape[2]
    K = A.shape[2] if transA == 0 else A.shape[1]
    a, b = complex(alpha), complex(beta)
    rc = lib.feast_zgemm_batched(int(transA), M, N, K, FeastZ(a.real, a.imag),
                                 C.c_void_p(A.data_ptr()), A.stride(1), A.stride(0),
                                 C.c_void_p(B.data_ptr()), B.stride(1), B.stride(0),
                                 FeastZ(b.real, b.imag), C.c_void_p(C_.data_ptr()), C_.stride(1),
                                 C_.stride(0), batch, _stream(stream))
    if rc != FEAST_OK:
        raise FeastError(rc, "feast_zgemm_batched")
    return C_


def zgetrf_batched(M, nb: int = 0, stream=None):
    """In-place LU of a (batch, n, n) complex128 tensor; returns (piv, info) int32 tensors."""
    import torch
    lib = load()
    batch, n = M.shape[0], M.shape[1]
    piv = torch.empty((batch, n), dtype=torch.int32, device=M.device)
    info = torch.empty((batch,), dtype=torch.int32, device=M.device)
    rc = lib.feast_zgetrf_batched(n, batch, C.c_void_p(M.data_ptr()), M.stride(1), M.stride(0),
                                  C.c_void_p(piv.data_ptr()), C.c_void_p(info.data_ptr()), nb,
                                  _stream(stream))
    if rc != FEAST_OK:
        raise FeastError(rc, "feast_zgetrf_batched")
    return piv, info


def zgetrs_batched(LU, piv, X, trans: int = 0, stream=None):
    return _zgetrs("feast_zgetrs_batched", LU, piv, X, trans, stream)


def zgetrs_batched_noalloc(LU, piv, X, trans: int = 0, stream=None):
    """As zgetrs_batched, with the library's fixed device scratch instead of
    allocations; asynchronous on the stream."""
    return _zgetrs("feast_zgetrs_batched_noalloc", LU, piv, X, trans, stream)


def _zgetrs(name, LU, piv, X, trans, stream):
    lib = load()
    batch, n = LU.shape[0], LU.shape[1]
    nrhs = X.shape[2]
    rc = getattr(lib, name)(n, nrhs, batch, C.c_void_p(LU.data_ptr()), LU.stride(1),
                            LU.stride(0), C.c_void_p(piv.data_ptr()), C.c_void_p(X.data_ptr()),
                            X.stride(1), X.stride(0), int(trans), _stream(stream))
    if rc != FEAST_OK:
        raise FeastError(rc, name)
    return X


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class BatchResult:
    lam: list              # per pencil: selected eigenvalues (numpy)
    X: list                # per pencil: torch tensor n x s (device)
    res: list              # per pencil: residuals r_i of eq. (5-1)
    err: np.ndarray
    flag: np.ndarray
    iters: np.ndarray
    info: dict


class Batch:
    """Many independent pencils of uneven order, factored and filtered in
    lockstep (grouped launches replayed from HIP graphs)."""

    def __init__(self, ns, ms, centers, radii, nodes: int, rule: int = TRAPEZOID,
                 eps: float = 1e-10, eta: float = 1e-3, max_iter: int = 20, prec: int = FP64,
                 max_sweeps: int = 6, nb: int = 0, batch_update: int = 0, stream=None):
        self.lib = load()
        self.ns = [int(x) for x in ns]
        self.ms = [int(x) for x in ms]
        P = len(self.ns)
        if len(self.ms) != P or len(centers) != P or len(radii) != P:
            raise ValueError("one n, m, center and radius per pencil")
        self.P = P
        self._c = (Contour * P)(*[contour(c, r, nodes, rule) for c, r in zip(centers, radii)])
        self.opts = default_opts()
        self.opts.eps, self.opts.eta, self.opts.max_iter = float(eps), float(eta), int(max_iter)
        self.opts.prec, self.opts.max_sweeps = int(prec), int(max_sweeps)
        self.opts.nb, self.opts.batch_update = int(nb), int(batch_update)
        self._stream_obj = stream
        self._h = C.c_void_p()
        n_arr = (C.c_int64 * P)(*self.ns)
        m_arr = (C.c_int64 * P)(*self.ms)
        rc = self.lib.feast_batch_create(C.byref(self._h), P, n_arr, m_arr, self._c,
                                         C.byref(self.opts), _stream(stream))
        if rc != FEAST_OK:
            raise FeastError(rc, "feast_batch_create failed")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.feast_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return self.lib.feast_batch_last_error(self._h).decode()

    def invalidate(self):
        self.lib.feast_batch_invalidate(self._h)

    def _mats(self, ts, rows, cols, name):
        ptrs = (C.c_void_p * self.P)()
        lds = (C.c_int64 * self.P)()
        if len(ts) != self.P:
            raise ValueError("%s: one tensor per pencil" % name)
        for i, t in enumerate(ts):
            p, ld = _dev(t, rows[i], cols[i], "%s[%d]" % (name, i))
            ptrs[i], lds[i] = p, ld
        return ptrs, lds

    def filter(self, As, Bs, Vs, sweeps: int = 0):
        """U_p = sum_j w_pj (z_pj B_p - A_p)^{-1} B_p V_p for every pencil."""
        import torch
        a, la = self._mats(As, self.ns, self.ns, "A")
        b, lb = self._mats(Bs, self.ns, self.ns, "B")
        v, lv = self._mats(Vs, self.ns, self.ms, "V")
        Us = [torch.empty((n, m), dtype=torch.complex128, device=Vs[0].device)
              for n, m in zip(self.ns, self.ms)]
        u, lu = self._mats(Us, self.ns, self.ms, "U")
        rc = self.lib.feast_batch_filter(self._h, a, la, b, lb, v, lv, u, lu, int(sweeps))
        if rc != FEAST_OK:
            raise FeastError(rc, self.last_error())
        return Us

    def solve(self, As, Bs, Vs) -> BatchResult:
        import torch
        P = self.P
        a, la = self._mats(As, self.ns, self.ns, "A")
        b, lb = self._mats(Bs, self.ns, self.ns, "B")
        v, lv = self._mats(Vs, self.ns, self.ms, "V")
        Xs = [torch.zeros((n, m), dtype=torch.complex128, device=Vs[0].device)
              for n, m in zip(self.ns, self.ms)]
        x, lx = self._mats(Xs, self.ns, self.ms, "X")
        lam = [np.zeros(m, dtype=np.complex128) for m in self.ms]
        res = [np.zeros(m, dtype=np.float64) for m in self.ms]
        hl = (C.c_void_p * P)(*[C.c_void_p(l.ctypes.data) for l in lam])
        hr = (C.c_void_p * P)(*[C.c_void_p(r.ctypes.data) for r in res])
        s_found = (C.c_int32 * P)()
        err = (C.c_double * P)()
        flag = (C.c_int32 * P)()
        iters = (C.c_int32 * P)()
        info = BatchInfo()
        rc = self.lib.feast_batch_solve(self._h, a, la, b, lb, v, lv, hl, x, lx, hr, s_found, err,
                                        flag, iters, C.byref(info))
        if rc != FEAST_OK:
            raise FeastError(rc, self.last_error())
        torch.cuda.current_stream().synchronize()
        k = list(s_found)
        return BatchResult(
            lam=[lam[i][:k[i]].copy() for i in range(P)],
            X=[Xs[i][:, :k[i]] for i in range(P)],
            res=[res[i][:k[i]].copy() for i in range(P)],
            err=np.array(list(err)), flag=np.array(list(flag)), iters=np.array(list(iters)),
            info={"iters": info.iters, "filters": info.filters,
                  "graph_launches": info.graph_launches, "factor": info.t_factor_ms,
                  "filter": info.t_filter_ms, "project": info.t_project_ms,
                  "host_eig": info.t_host_eig_ms, "total": info.t_total_ms})
