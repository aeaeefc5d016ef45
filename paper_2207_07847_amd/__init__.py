"""Python binding of liblapgpu.so, the MI355X MSP-preconditioned Laplacian
solver (Hu & Lin, arXiv 2207.07847).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Functions carry the C names of include/lap.h.  Device
buffers are passed as integer addresses (``tensor.data_ptr()``) and streams
as integer handles (``torch.cuda.current_stream().cuda_stream``); PyTorch is
used by callers for device memory and streams only.

Importing this module raises if the compiled library is missing: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblapgpu.so")

LAP_OK, LAP_EINVAL, LAP_EDISCONNECTED, LAP_ENOMEM, LAP_EDEVICE, LAP_ENOCONV, \
    LAP_EBREAKDOWN, LAP_EUNSUPPORTED = range(8)
LAP_PREC_MSP, LAP_PREC_PEGP, LAP_PREC_NONE, LAP_PREC_OFFTREE, LAP_PREC_SPANNING = 0, 1, 2, 3, 4
LAP_FP64 = 0
LAP_MIXED_FP32_FP64 = 1
LAP_FLAG_HOST_ONLY = 1
LAP_FLAG_FGMRES = 4
LAP_FLAG_DEVICE_SETUP = 8
LAP_FLAG_PARALLEL_MATCHING = 16
LAP_FLAG_MULTI_RHS = 2
LAP_MAX_LEVELS = 64
LAP_KERNEL_SPMV, LAP_KERNEL_UPDATE, LAP_KERNEL_DOWN0, LAP_KERNEL_PRECOND, LAP_KERNEL_ITER = range(5)
LAP_KERNEL_BLOCK_SPMM, LAP_KERNEL_BLOCK_ITER, LAP_KERNEL_PEGP_OP = 5, 6, 7


class lap_graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("u", C.POINTER(C.c_int64)),
                ("v", C.POINTER(C.c_int64)), ("w", C.POINTER(C.c_double))]


class lap_params(C.Structure):
    _fields_ = [("mu", C.c_double), ("max_levels", C.c_int32), ("n_top", C.c_int32),
                ("mwm_seed", C.c_uint64), ("precond", C.c_int32), ("precision", C.c_int32),
                ("max_iter", C.c_int32), ("flags", C.c_uint32), ("offtree_frac", C.c_double)]


class lap_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("refinements", C.c_int32),
                ("relres_true", C.c_double), ("relres_recursive", C.c_double),
                ("seconds", C.c_double), ("status", C.c_int32), ("pad", C.c_int32)]


class lap_hierarchy_desc(C.Structure):
    _fields_ = [("nlev", C.c_int32), ("tail_level", C.c_int32),
                ("sizes", C.c_int64 * LAP_MAX_LEVELS), ("ntilde", C.c_int64),
                ("nnz", C.c_int64), ("device_bytes", C.c_int64), ("setup_seconds", C.c_double),
                ("mm_chunk", C.c_int32 * 2), ("mm_grid", C.c_int32 * 2),
                ("mm_seg", C.c_int32 * 2), ("mm_tune_seconds", C.c_double),
                ("spmv_fused", C.c_int32), ("pegp_operator_n", C.c_int32)]


class lap_request_result(C.Structure):
    _fields_ = [("tag", C.c_int64), ("graph", C.c_int32), ("nrhs", C.c_int32),
                ("status", C.c_int32), ("iterations_max", C.c_int32),
                ("relres_max", C.c_double), ("queue_seconds", C.c_double),
                ("total_seconds", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def _load():
    # Device buffers come from torch, so the library must run on the same HIP
    # runtime instance: torch ships its own libamdhip64.so.7; importing torch
    # first makes the dynamic loader resolve the library's libamdhip64.so.7 to
    # that copy instead of mapping a second runtime into the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2207_07847_amd.build")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.lap_default_params.argtypes = [C.POINTER(lap_params)]
    L.lap_setup.argtypes = [C.POINTER(lap_graph), C.POINTER(lap_params), vp, C.POINTER(vp)]
    L.lap_solve.argtypes = [vp, vp, vp, C.c_int32, C.c_int64, C.c_double,
                            C.POINTER(lap_solve_info), vp]
    L.lap_set_precision.argtypes = [vp, C.c_int32]
    L.lap_apply_laplacian.argtypes = [vp, vp, vp, vp]
    L.lap_apply_laplacian_noalloc.argtypes = [vp, vp, vp, vp]
    L.lap_apply_precond.argtypes = [vp, vp, vp, vp]
    L.lap_hierarchy_info.argtypes = [vp, C.POINTER(lap_hierarchy_desc)]
    L.lap_export_level.argtypes = [vp, C.c_int32, vp, vp]
    L.lap_export_graph.argtypes = [vp, C.c_int32, vp, vp, vp]
    L.lap_export_offtree.argtypes = [vp, C.POINTER(C.c_int64), vp, vp, vp, vp, vp]
    L.lap_profile_kernel.argtypes = [vp, C.c_int32, C.c_int32, vp, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
    L.lap_estimate_spectrum.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_int32), vp]
    L.lap_select_mu.argtypes = [C.POINTER(lap_graph), C.POINTER(lap_params), vp, C.c_int32, vp,
                                C.c_int32, vp, C.POINTER(C.c_int32), vp]
    L.lap_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
    L.lap_set_allocator.restype = C.c_int
    L.lap_free.argtypes = [vp]
    L.lap_free.restype = None
    L.lap_server_create.argtypes = [C.c_int64, C.POINTER(vp)]
    L.lap_server_add.argtypes = [vp, vp, C.POINTER(C.c_int32)]
    L.lap_server_submit.argtypes = [vp, C.c_int32, vp, vp, C.c_int32, C.c_double, C.c_int64]
    L.lap_server_poll.argtypes = [vp, C.POINTER(lap_request_result), C.c_int32, C.c_int32,
                                  C.POINTER(C.c_int32)]
    L.lap_server_destroy.argtypes = [vp]
    L.lap_server_destroy.restype = None
    for f in ("lap_server_create", "lap_server_add", "lap_server_submit", "lap_server_poll"):
        getattr(L, f).restype = C.c_int
    L.lap_last_error.argtypes = []
    L.lap_last_error.restype = C.c_char_p
    L.lap_status_str.argtypes = [C.c_int]
    L.lap_status_str.restype = C.c_char_p
    for f in ("lap_default_params", "lap_setup", "lap_solve", "lap_set_precision",
              "lap_apply_laplacian", "lap_apply_laplacian_noalloc",
              "lap_apply_precond", "lap_hierarchy_info", "lap_export_level", "lap_export_graph",
              "lap_export_offtree",
              "lap_profile_kernel", "lap_estimate_spectrum", "lap_select_mu"):
        getattr(L, f).restype = C.c_int
    return L


_lib = _load()


class LapError(RuntimeError):
    def __init__(self, status, what=""):
        extra = lap_last_error() if status == LAP_EDEVICE else ""
        super().__init__(f"{what}: {lap_status_str(status)} {extra}".rstrip())
        self.status = status


def lap_last_error() -> str:
    return _lib.lap_last_error().decode()


def lap_status_str(status: int) -> str:
    return _lib.lap_status_str(int(status)).decode()


def lap_default_params(**overrides) -> lap_params:
    p = lap_params()
    _lib.lap_default_params(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _graph(n, u, v, w):
    """(lap_graph, the arrays it points into, which must outlive it)."""
    u = np.ascontiguousarray(u, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.int64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    g = lap_graph(int(n), len(u), u.ctypes.data_as(C.POINTER(C.c_int64)),
                  v.ctypes.data_as(C.POINTER(C.c_int64)), w.ctypes.data_as(C.POINTER(C.c_double)))
    return g, (u, v, w)


def lap_setup(n, u, v, w, params: lap_params | None = None, stream=0):
    """Host setup + upload.  u, v, w: host arrays (copied during the call).
    Returns an opaque handle (int); raises LapError on a non-OK status."""
    g, keep = _graph(n, u, v, w)
    p = params if params is not None else lap_default_params()
    h = C.c_void_p()
    st = _lib.lap_setup(C.byref(g), C.byref(p), C.c_void_p(stream or 0), C.byref(h))
    if st != LAP_OK:
        raise LapError(st, "lap_setup")
    return h.value


def lap_solve(h, b_ptr: int, x_ptr: int, n: int, tol: float, nrhs: int = 1, ld: int | None = None,
              stream=0):
    """Returns (status, [info dict per column])."""
    info = (lap_solve_info * nrhs)()
    st = _lib.lap_solve(C.c_void_p(h), C.c_void_p(b_ptr), C.c_void_p(x_ptr), int(nrhs),
                        int(ld if ld is not None else n), float(tol), info, C.c_void_p(stream or 0))
    out = [dict(iterations=i.iterations, refinements=i.refinements, relres_true=i.relres_true,
                relres_recursive=i.relres_recursive, seconds=i.seconds, status=i.status)
           for i in info]
    return st, out


def lap_set_precision(h, precision: int) -> int:
    return _lib.lap_set_precision(C.c_void_p(h), int(precision))


def lap_apply_laplacian_noalloc(h, x_ptr: int, y_ptr: int, stream=0) -> int:
    return _lib.lap_apply_laplacian_noalloc(C.c_void_p(h), C.c_void_p(x_ptr),
                                            C.c_void_p(y_ptr), C.c_void_p(stream or 0))


def lap_apply_laplacian(h, x_ptr: int, y_ptr: int, stream=0) -> int:
    return _lib.lap_apply_laplacian(C.c_void_p(h), C.c_void_p(x_ptr), C.c_void_p(y_ptr),
                                    C.c_void_p(stream or 0))


def lap_apply_precond(h, r_ptr: int, z_ptr: int, stream=0) -> int:
    return _lib.lap_apply_precond(C.c_void_p(h), C.c_void_p(r_ptr), C.c_void_p(z_ptr),
                                  C.c_void_p(stream or 0))


def lap_hierarchy_info(h) -> dict:
    d = lap_hierarchy_desc()
    st = _lib.lap_hierarchy_info(C.c_void_p(h), C.byref(d))
    if st != LAP_OK:
        raise LapError(st, "lap_hierarchy_info")
    return dict(nlev=d.nlev, tail_level=d.tail_level, sizes=list(d.sizes[:d.nlev]),
                ntilde=d.ntilde, nnz=d.nnz, device_bytes=d.device_bytes,
                setup_seconds=d.setup_seconds, mm_chunk=list(d.mm_chunk),
                mm_grid=list(d.mm_grid), mm_seg=list(d.mm_seg),
                mm_tune_seconds=d.mm_tune_seconds, spmv_fused=bool(d.spmv_fused),
                pegp_operator_n=d.pegp_operator_n)


def lap_export_level(h, level: int, size: int):
    agg = np.empty(size, dtype=np.int64)
    mt = np.empty(size, dtype=np.int8)
    st = _lib.lap_export_level(C.c_void_p(h), int(level), agg.ctypes.data, mt.ctypes.data)
    if st != LAP_OK:
        raise LapError(st, "lap_export_level")
    return agg, mt.astype(bool)


def lap_export_graph(h, level: int, size: int):
    ptr = np.empty(size + 1, dtype=np.int64)
    st = _lib.lap_export_graph(C.c_void_p(h), int(level), ptr.ctypes.data, None, None)
    if st != LAP_OK:
        raise LapError(st, "lap_export_graph")
    col = np.empty(int(ptr[-1]), dtype=np.int64)
    w = np.empty(int(ptr[-1]), dtype=np.float64)
    _lib.lap_export_graph(C.c_void_p(h), int(level), ptr.ctypes.data, col.ctypes.data,
                          w.ctypes.data)
    return ptr, col, w


def lap_export_offtree(h):
    """Off-tree edges of a LAP_PREC_OFFTREE or LAP_PREC_SPANNING hierarchy: dict of arrays a, b
    (expanded indices in the levels' own numbering), w, stretch, kept."""
    cnt = C.c_int64()
    st = _lib.lap_export_offtree(C.c_void_p(h), C.byref(cnt), None, None, None, None, None)
    if st != LAP_OK:
        raise LapError(st, "lap_export_offtree")
    k = cnt.value
    out = dict(a=np.empty(k, np.int64), b=np.empty(k, np.int64), w=np.empty(k),
               stretch=np.empty(k), kept=np.empty(k, np.int8))
    _lib.lap_export_offtree(C.c_void_p(h), C.byref(cnt), out["a"].ctypes.data,
                            out["b"].ctypes.data, out["w"].ctypes.data,
                            out["stretch"].ctypes.data, out["kept"].ctypes.data)
    return out


def lap_profile_kernel(h, kernel: int, reps: int, stream=0):
    """Returns (avg_ms per launch, algorithmic bytes per launch)."""
    ms = C.c_double()
    by = C.c_double()
    st = _lib.lap_profile_kernel(C.c_void_p(h), int(kernel), int(reps), C.c_void_p(stream or 0),
                                 C.byref(ms), C.byref(by))
    if st != LAP_OK:
        raise LapError(st, "lap_profile_kernel")
    return ms.value, by.value


def lap_estimate_spectrum(h, b_ptr: int, steps: int, stream=0):
    """(status, lambda_min, lambda_max, steps taken) of M L on range(L)."""
    lo, hi, k = C.c_double(), C.c_double(), C.c_int32()
    st = _lib.lap_estimate_spectrum(C.c_void_p(h), C.c_void_p(b_ptr), int(steps), C.byref(lo),
                                    C.byref(hi), C.byref(k), C.c_void_p(stream or 0))
    return st, lo.value, hi.value, k.value


def lap_select_mu(n, u, v, w, mus, b_ptr: int, steps: int, params: lap_params | None = None,
                  stream=0):
    """(status, best index, estimated kappa per candidate)."""
    g, keep = _graph(n, u, v, w)
    p = params if params is not None else lap_default_params()
    m = np.ascontiguousarray(mus, dtype=np.float64)
    kap = np.zeros(len(m))
    best = C.c_int32(-1)
    st = _lib.lap_select_mu(C.byref(g), C.byref(p), m.ctypes.data, len(m), C.c_void_p(b_ptr),
                            int(steps), kap.ctypes.data, C.byref(best), C.c_void_p(stream or 0))
    return st, best.value, kap


# every callback pair ever registered stays referenced: a hierarchy keeps
# calling the pair it was set up with until lap_free
_allocators = []


def lap_set_allocator(alloc=None, free=None) -> int:
    """Device allocator of later lap_setup calls: alloc(nbytes) -> device
    pointer (int, 0 on failure), free(ptr) -> None.  No arguments restores
    hipMalloc / hipFree."""
    if alloc is None and free is None:
        return _lib.lap_set_allocator(C.cast(None, ALLOC_FN), C.cast(None, FREE_FN), None)
    if alloc is None or free is None:
        return LAP_EINVAL
    a = ALLOC_FN(lambda nbytes, ctx: alloc(int(nbytes)) or None)
    f = FREE_FN(lambda ptr, ctx: free(int(ptr)))
    _allocators.append((a, f))
    return _lib.lap_set_allocator(a, f, None)


def use_torch_allocator(device=None) -> int:
    """Route the device memory of later hierarchies through torch's caching
    allocator (on `device`, default the current one)."""
    import torch
    dev = torch.cuda.current_device() if device is None else device

    def alloc(nbytes):
        try:
            return torch.cuda.caching_allocator_alloc(nbytes, dev)
        except RuntimeError:
            return 0

    def free(ptr):
        torch.cuda.caching_allocator_delete(ptr)

    return lap_set_allocator(alloc, free)


def lap_free(h) -> None:
    if h:
        _lib.lap_free(C.c_void_p(h))


def lap_server_create(hbm_budget_bytes: int = 0):
    srv = C.c_void_p()
    st = _lib.lap_server_create(int(hbm_budget_bytes), C.byref(srv))
    if st != LAP_OK:
        raise LapError(st, "lap_server_create")
    return srv.value


def lap_server_add(srv, h) -> int:
    gid = C.c_int32()
    st = _lib.lap_server_add(C.c_void_p(srv), C.c_void_p(h), C.byref(gid))
    if st != LAP_OK:
        raise LapError(st, "lap_server_add")
    return gid.value


def lap_server_submit(srv, graph: int, b_ptr: int, x_ptr: int, nrhs: int, tol: float,
                      tag: int) -> int:
    """b_ptr, x_ptr: host addresses (e.g. numpy .ctypes.data), column-major,
    kept alive by the caller until the result is polled."""
    return _lib.lap_server_submit(C.c_void_p(srv), int(graph), C.c_void_p(b_ptr),
                                  C.c_void_p(x_ptr), int(nrhs), float(tol), int(tag))


def lap_server_poll(srv, max_results: int = 256, wait_ms: int = 0) -> list:
    out = (lap_request_result * max(1, max_results))()
    cnt = C.c_int32()
    st = _lib.lap_server_poll(C.c_void_p(srv), out, int(max_results), int(wait_ms),
                              C.byref(cnt))
    if st != LAP_OK:
        raise LapError(st, "lap_server_poll")
    return [dict(tag=o.tag, graph=o.graph, nrhs=o.nrhs, status=o.status,
                 iterations_max=o.iterations_max, relres_max=o.relres_max,
                 queue_seconds=o.queue_seconds, total_seconds=o.total_seconds)
            for o in out[:cnt.value]]


def lap_server_destroy(srv) -> None:
    if srv:
        _lib.lap_server_destroy(C.c_void_p(srv))
