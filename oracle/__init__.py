"""FP64 oracle for the multilevel-sparsifier Laplacian solve (Hu & Lin,
arXiv 2207.07847).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the GPU library (``paper_2207_07847_amd``) and never imports it.

Three parts:
  * ``liblapref.so`` (``lapref.c``): plain sequential C, FP64 - graph CSR,
    maximal-weighted-matching hierarchy, coarse graphs, the MSP sparsifier
    T~ solved by Gaussian elimination, and preconditioned CG;
  * ``oracle.dense``: explicit dense matrices of the paper's definitions for
    tiny graphs (P(mu), L_G~, H~, T~, pseudo-inverses, condition numbers);
  * ``oracle.pegp``: the PEGP preconditioner with a sparse direct solve.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblapref.so")
_lib = None

OK, EINVAL, EDISCONNECTED, ENOMEM, ENOCONV, EBREAKDOWN = 0, 1, 2, 3, 5, 6

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
PRECOND_FN = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double))


class _PcgInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32),
                ("relres_recursive", C.c_double), ("relres_true", C.c_double),
                ("restarts", C.c_int32), ("pad", C.c_int32)]


def build(force: bool = True) -> str:
    """Compile lapref.c into liblapref.so with gcc."""
    src = os.path.join(_HERE, "lapref.c")
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    L = C.CDLL(_LIB_PATH)
    vp = C.c_void_p
    L.lr_csr_build.argtypes = [C.c_int64, C.c_int64, _i64p, _i64p, _f64p, C.POINTER(vp)]
    L.lr_csr_build.restype = C.c_int
    L.lr_csr_free.argtypes = [vp]
    L.lr_connected.argtypes = [vp]
    L.lr_connected.restype = C.c_int
    L.lr_lap_apply.argtypes = [vp, _f64p, _f64p]
    L.lr_mwm.argtypes = [vp, vp, _i64p, _i8p]
    L.lr_mwm.restype = C.c_int64
    L.lr_hier_build.argtypes = [vp, C.c_int32, C.c_int64, C.c_uint64, C.POINTER(vp)]
    L.lr_hier_build_ex.argtypes = [vp, C.c_int32, C.c_int64, C.c_uint64, C.c_int32,
                                   C.POINTER(vp)]
    L.lr_hier_build_ex.restype = C.c_int
    L.lr_greedy_match.argtypes = [vp, _i64p, _i8p]
    L.lr_greedy_match.restype = C.c_int64
    L.lr_hier_build.restype = C.c_int
    L.lr_hier_free.argtypes = [vp]
    L.lr_hier_nlev.argtypes = [vp]
    L.lr_hier_nlev.restype = C.c_int32
    L.lr_hier_nk.argtypes = [vp, C.c_int32]
    L.lr_hier_nk.restype = C.c_int64
    L.lr_hier_agg.argtypes = [vp, C.c_int32, _i64p, _i8p]
    L.lr_hier_level_nnz.argtypes = [vp, C.c_int32]
    L.lr_hier_level_nnz.restype = C.c_int64
    L.lr_hier_level_csr.argtypes = [vp, C.c_int32, _i64p, _i64p, _f64p]
    L.lr_hier_ntilde.argtypes = [vp]
    L.lr_hier_ntilde.restype = C.c_int64
    L.lr_restrict_mu.argtypes = [vp, C.c_double, _f64p, _f64p]
    L.lr_prolong_mu.argtypes = [vp, C.c_double, _f64p, _f64p]
    L.lr_msp_edges.argtypes = [vp, C.c_double, C.POINTER(C.c_int64),
                               C.POINTER(C.POINTER(C.c_int64)),
                               C.POINTER(C.POINTER(C.c_int64)),
                               C.POINTER(C.POINTER(C.c_double))]
    L.lr_msp_edges.restype = C.c_int
    L.lr_free.argtypes = [vp]
    L.lr_msp_factor.argtypes = [vp, C.c_double, C.POINTER(vp)]
    L.lr_msp_factor.restype = C.c_int
    L.lr_msp_free.argtypes = [vp]
    L.lr_msp_fill.argtypes = [vp]
    L.lr_msp_fill.restype = C.c_int64
    L.lr_msp_apply.argtypes = [vp, _f64p, _f64p]
    L.lr_msp_solve_expanded.argtypes = [vp, _f64p, _f64p]
    L.lr_msp_solve_expanded.restype = None
    L.lr_pcg.argtypes = [vp, vp, vp, _f64p, C.c_double, C.c_int32, _f64p,
                         C.POINTER(_PcgInfo), vp]
    L.lr_pcg.restype = C.c_int
    L.lr_pcg_noisy.argtypes = [vp, vp, vp, _f64p, C.c_double, C.c_int32, _f64p,
                               C.POINTER(_PcgInfo), vp, C.c_double, C.c_uint64]
    L.lr_pcg_noisy.restype = C.c_int
    L.lr_pcg_ex.argtypes = [vp, vp, vp, _f64p, C.c_double, C.c_int32, _f64p,
                            C.POINTER(_PcgInfo), vp, C.c_double, C.c_uint64, C.c_int32]
    L.lr_pcg_ex.restype = C.c_int
    _lib = L
    return L


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


class Graph:
    """Symmetric CSR of an undirected weighted edge list (Sec. 2.1)."""

    def __init__(self, n, u, v, w):
        L = lib()
        self._h = C.c_void_p()
        u = np.ascontiguousarray(u, dtype=np.int64)
        v = np.ascontiguousarray(v, dtype=np.int64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        rc = L.lr_csr_build(int(n), len(u), u, v, w, C.byref(self._h))
        if rc != OK:
            raise OracleError(rc, "graph")
        self.n = int(n)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lr_csr_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def connected(self) -> bool:
        return bool(lib().lr_connected(self._h))

    def apply(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        lib().lr_lap_apply(self._h, x, y)
        return y

    def mwm(self, order=None):
        agg = np.empty(self.n, dtype=np.int64)
        mt = np.empty(self.n, dtype=np.int8)
        if order is None:
            nc = lib().lr_mwm(self._h, None, agg, mt)
        else:
            order = np.ascontiguousarray(order, dtype=np.int64)
            nc = lib().lr_mwm(self._h, order.ctypes.data, agg, mt)
        return int(nc), agg, mt.astype(bool)


MATCHINGS = {"visit": 0, "greedy": 1}


class Hierarchy:
    """Aggregation hierarchy over a Graph: matching "visit" is the
    visit-order matching of Sec. 2.2 (lr_mwm), "greedy" the greedy matching
    by edge weight of a parallel setup (lr_greedy_match)."""

    def __init__(self, g: Graph, max_levels=0, n_top=2, seed=0, matching="visit"):
        self._h = C.c_void_p()
        rc = lib().lr_hier_build_ex(g.handle, int(max_levels), int(n_top),
                                    int(seed), MATCHINGS[matching], C.byref(self._h))
        if rc != OK:
            raise OracleError(rc, "hierarchy")
        self.g = g

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lr_hier_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def nlev(self):
        return int(lib().lr_hier_nlev(self._h))

    @property
    def sizes(self):
        return [int(lib().lr_hier_nk(self._h, k)) for k in range(self.nlev)]

    @property
    def ntilde(self):
        return int(lib().lr_hier_ntilde(self._h))

    def agg(self, k):
        n = lib().lr_hier_nk(self._h, k)
        a = np.empty(n, dtype=np.int64)
        mt = np.empty(n, dtype=np.int8)
        lib().lr_hier_agg(self._h, k, a, mt)
        return a, mt.astype(bool)

    def aggs(self):
        return [self.agg(k)[0] for k in range(self.nlev - 1)]

    def level_csr(self, k):
        n = lib().lr_hier_nk(self._h, k)
        nnz = lib().lr_hier_level_nnz(self._h, k)
        ptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int64)
        w = np.empty(nnz, dtype=np.float64)
        lib().lr_hier_level_csr(self._h, k, ptr, col, w)
        return ptr, col, w

    def restrict_mu(self, mu, r):
        out = np.empty(self.ntilde)
        lib().lr_restrict_mu(self._h, float(mu), np.ascontiguousarray(r, dtype=np.float64), out)
        return out

    def prolong_mu(self, mu, yt):
        out = np.empty(self.sizes[0])
        lib().lr_prolong_mu(self._h, float(mu), np.ascontiguousarray(yt, dtype=np.float64), out)
        return out

    def msp_edges(self, mu):
        ne = C.c_int64()
        pu = C.POINTER(C.c_int64)()
        pv = C.POINTER(C.c_int64)()
        pw = C.POINTER(C.c_double)()
        lib().lr_msp_edges(self._h, float(mu), C.byref(ne), C.byref(pu), C.byref(pv), C.byref(pw))
        m = ne.value
        u = np.ctypeslib.as_array(pu, shape=(max(m, 1),))[:m].copy()
        v = np.ctypeslib.as_array(pv, shape=(max(m, 1),))[:m].copy()
        w = np.ctypeslib.as_array(pw, shape=(max(m, 1),))[:m].copy()
        for p in (pu, pv, pw):
            lib().lr_free(C.cast(p, C.c_void_p))
        return u, v, w


class MSP:
    """Factored MSP sparsifier: apply(r) = P(mu) L_T~^+ P(mu)^T r, mean-free."""

    def __init__(self, h: Hierarchy, mu):
        self._f = C.c_void_p()
        rc = lib().lr_msp_factor(h.handle, float(mu), C.byref(self._f))
        if rc != OK:
            raise OracleError(rc, "msp")
        self.h = h
        self.mu = float(mu)
        self.n = h.sizes[0]

    def __del__(self):
        if getattr(self, "_f", None) and _lib is not None:
            _lib.lr_msp_free(self._f)
            self._f = None

    @property
    def fill(self):
        return int(lib().lr_msp_fill(self._f))

    def apply(self, r):
        z = np.empty(self.n)
        lib().lr_msp_apply(self._f, np.ascontiguousarray(r, dtype=np.float64), z)
        return z

    def solve_expanded(self, bt):
        """Grounded solve of L_T~ y~ = b~ in the expanded space (Sec. 3.3)."""
        y = np.empty(self.h.ntilde)
        lib().lr_msp_solve_expanded(self._f, np.ascontiguousarray(bt, dtype=np.float64), y)
        return y


def greedy_match(g: Graph):
    """(agg, matched, nc) of lr_greedy_match on the fine level of g."""
    agg = np.empty(g.n, dtype=np.int64)
    mt = np.empty(g.n, dtype=np.int8)
    nc = lib().lr_greedy_match(g.handle, agg, mt)
    return agg, mt, int(nc)


def iteration_band(g: Graph, b, tol, maxit, precond, seeds=8, noise=4e-16):
    """(min, max) iteration count over the unperturbed run and `seeds` runs of
    the rounding model (relative noise `noise` on L p and M r)."""
    its = [pcg(g, b, tol, maxit, precond).iterations]
    its += [pcg(g, b, tol, maxit, precond, noise=noise, seed=s + 1).iterations
            for s in range(seeds)]
    return min(its), max(its)


class PcgResult:
    def __init__(self, x, info, hist):
        self.x = x
        self.iterations = int(info.iterations)
        self.status = int(info.status)
        self.relres_recursive = float(info.relres_recursive)
        self.relres_true = float(info.relres_true)
        self.restarts = int(info.restarts)
        self.hist = hist[: self.iterations + 1]


MAX_RESTARTS = 3   # residual replacements after a converged recurrence (Sec. 4 stop rule)


def pcg(g: Graph, b, tol=1e-8, maxit=1000, precond=None, noise=0.0, seed=0,
        restarts=MAX_RESTARTS):
    """PCG on L_G x = b.  precond: None (plain CG), an MSP, or a callable
    r -> z on numpy arrays (e.g. the PEGP of oracle.pegp).  noise > 0 runs
    the rounding model of lr_pcg_noisy.  restarts: residual replacements
    allowed when the recurrence converges with a true residual above tol
    (lr_pcg_ex)."""
    L = lib()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(g.n)
    info = _PcgInfo()
    hist = np.zeros(int(maxit) + 1)
    keep = None
    if precond is None:
        fn, ctx = None, None
    elif isinstance(precond, MSP):
        fn, ctx = C.cast(L.lr_msp_apply, C.c_void_p), precond._f
    else:
        n = g.n

        def _cb(_ctx, rp, zp):
            r = np.ctypeslib.as_array(rp, shape=(n,))
            z = np.ctypeslib.as_array(zp, shape=(n,))
            z[:] = precond(r.copy())

        keep = PRECOND_FN(_cb)
        fn, ctx = C.cast(keep, C.c_void_p), None
    L.lr_pcg_ex(g.handle, fn, ctx, b, float(tol), int(maxit), x, C.byref(info),
                hist.ctypes.data, float(noise), int(seed), int(restarts))
    del keep
    return PcgResult(x, info, hist)
