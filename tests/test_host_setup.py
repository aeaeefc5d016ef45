"""CPU tests of the library's host side: the C ABI surface, the integer
outputs of the aggregation hierarchy (bit-exact against the oracle) and the
coarse graphs (exact FP64 equality, since both sides sum the same fine
weights in the same stated order), and argument/graph validation."""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lap():
    import paper_2207_07847_amd as lap
    return lap


def test_library_exports_every_declared_symbol():
    """Every function declared in include/*.h is exported by liblapgpu.so."""
    import ctypes
    lap = _lap()
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            src = open(os.path.join(inc, fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(lap_[a-z_]+)\s*\(", src))
    assert len(names) >= 10
    dll = ctypes.CDLL(lap.LIB_PATH)
    for nm in sorted(names):
        assert hasattr(dll, nm), nm


def _graphs():
    out = []
    out.append(("grid2d_17x9", W.grid2d(17, 9), None))
    out.append(("grid3d_9", W.grid3d(9), "loguniform"))
    out.append(("ring_101", W.ring(101), None))
    out.append(("er_500", W.erdos_renyi(500, 6, 3), "uniform"))
    out.append(("ws_300", W.watts_strogatz(300, 4, 0.1, 4), "loguniform"))
    out.append(("chunglu_3000", W.chung_lu(3000, 8.0, 2.1, 5), "uniform"))
    out.append(("rmat_10", W.rmat(10, 8, seed=6), "uniform"))
    out.append(("path_37", W.path(37), None))
    out.append(("complete_9", W.complete(9), None))
    return out


def _weights(kind, m, seed):
    if kind is None:
        return W.unit_weights(m)
    if kind == "loguniform":
        return W.loguniform_weights(m, seed)
    return W.uniform01_weights(m, seed)


@pytest.mark.parametrize("seed", [0, 12345])
@pytest.mark.parametrize("case", range(9))
def test_hierarchy_bit_exact_vs_oracle(oracle_lib, case, seed):
    """Level sizes, aggregate ids, matched flags and coarse graphs equal the
    oracle's exactly (integer outputs bit for bit, FP64 weights exactly)."""
    from oracle import Graph, Hierarchy
    lap = _lap()
    name, (n, u, v), kind = _graphs()[case]
    w = _weights(kind, len(u), 100 + case)
    p = lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY, mwm_seed=seed)
    h = lap.lap_setup(n, u, v, w, p)
    try:
        info = lap.lap_hierarchy_info(h)
        H = Hierarchy(Graph(n, u, v, w), seed=seed)
        assert info["sizes"] == H.sizes, name
        assert info["ntilde"] == H.ntilde
        for k in range(info["nlev"] - 1):
            a, m = lap.lap_export_level(h, k, info["sizes"][k])
            a2, m2 = H.agg(k)
            np.testing.assert_array_equal(a, a2)
            np.testing.assert_array_equal(m, m2)
        for k in range(info["nlev"]):
            pt, c, ww = lap.lap_export_graph(h, k, info["sizes"][k])
            pt2, c2, w2 = H.level_csr(k)
            np.testing.assert_array_equal(pt, pt2)
            np.testing.assert_array_equal(c, c2)
            np.testing.assert_array_equal(ww, w2)
    finally:
        lap.lap_free(h)


@pytest.mark.parametrize("max_levels", [2, 3])
def test_limited_levels_bit_exact(oracle_lib, max_levels):
    """level = 2 (Sec. 4.1) and other caps: same hierarchy as the oracle."""
    from oracle import Graph, Hierarchy
    lap = _lap()
    n, u, v = W.grid2d(32)
    w = W.unit_weights(len(u))
    p = lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY, max_levels=max_levels)
    h = lap.lap_setup(n, u, v, w, p)
    try:
        info = lap.lap_hierarchy_info(h)
        assert info["sizes"] == Hierarchy(Graph(n, u, v, w), max_levels=max_levels).sizes
        assert info["nlev"] == max_levels
    finally:
        lap.lap_free(h)


def test_parallel_edges_merged_in_input_order(oracle_lib):
    from oracle import Graph, Hierarchy
    lap = _lap()
    rng = np.random.default_rng(0)
    n, u, v = W.erdos_renyi(200, 5, 1)
    dup = rng.integers(0, len(u), 150)
    u2 = np.concatenate([u, v[dup]])
    v2 = np.concatenate([v, u[dup]])
    w2 = rng.random(len(u2)) + 0.1
    h = lap.lap_setup(n, u2, v2, w2, lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY))
    try:
        pt, c, ww = lap.lap_export_graph(h, 0, n)
        pt2, c2, w2o = Hierarchy(Graph(n, u2, v2, w2)).level_csr(0)
        np.testing.assert_array_equal(ww, w2o)
    finally:
        lap.lap_free(h)


@pytest.mark.parametrize("bad", ["selfloop", "range", "zero", "neg", "nan", "inf", "n1"])
def test_invalid_graph(bad):
    lap = _lap()
    n, u, v = 4, np.array([0, 1, 2]), np.array([1, 2, 3])
    w = np.ones(3)
    if bad == "selfloop":
        v = np.array([1, 2, 2])
    elif bad == "range":
        v = np.array([1, 2, 4])
    elif bad == "zero":
        w = np.array([1.0, 0.0, 1.0])
    elif bad == "neg":
        w = np.array([1.0, -2.0, 1.0])
    elif bad == "nan":
        w = np.array([1.0, np.nan, 1.0])
    elif bad == "inf":
        w = np.array([1.0, np.inf, 1.0])
    elif bad == "n1":
        n = 1
    with pytest.raises(lap.LapError) as e:
        lap.lap_setup(n, u, v, w, lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY))
    assert e.value.status == lap.LAP_EINVAL


def test_disconnected_graph():
    lap = _lap()
    with pytest.raises(lap.LapError) as e:
        lap.lap_setup(4, [0, 2], [1, 3], [1.0, 1.0],
                      lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY))
    assert e.value.status == lap.LAP_EDISCONNECTED


@pytest.mark.parametrize("field,value,code", [
    ("mu", 0.0, 1), ("mu", 1.0, 1), ("mu", -0.5, 1), ("n_top", 1, 1),
    ("precond", 9, 1), ("precision", 3, 1), ("max_iter", -1, 1),
])
def test_invalid_params(field, value, code):
    lap = _lap()
    n, u, v = W.grid2d(6)
    p = lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY)
    setattr(p, field, value)
    with pytest.raises(lap.LapError) as e:
        lap.lap_setup(n, u, v, np.ones(len(u)), p)
    assert e.value.status == code


def test_pegp_setup_limits():
    """PEGP: FP64 single solves only; the expanded system must fit one
    workgroup's LDS (host-only setups build and factor it)."""
    lap = _lap()
    n, u, v = W.grid2d(16)
    w = np.ones(len(u))
    p = lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY, precond=lap.LAP_PREC_PEGP,
                               mu=1 / 16)
    h = lap.lap_setup(n, u, v, w, p)
    assert lap.lap_hierarchy_info(h)["ntilde"] == 510
    lap.lap_free(h)
    for extra in (dict(precision=lap.LAP_MIXED_FP32_FP64),
                  dict(flags=lap.LAP_FLAG_HOST_ONLY | lap.LAP_FLAG_MULTI_RHS)):
        q = lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY, precond=lap.LAP_PREC_PEGP)
        for k, val in extra.items():
            setattr(q, k, val)
        with pytest.raises(lap.LapError) as e:
            lap.lap_setup(n, u, v, w, q)
        assert e.value.status == lap.LAP_EUNSUPPORTED
    n, u, v = W.grid2d(128)        # 32766 expanded nodes: beyond the LDS solve
    with pytest.raises(lap.LapError) as e:
        lap.lap_setup(n, u, v, np.ones(len(u)), p)
    assert e.value.status == lap.LAP_EUNSUPPORTED


def test_host_only_refuses_device_calls():
    lap = _lap()
    n, u, v = W.grid2d(6)
    h = lap.lap_setup(n, u, v, np.ones(len(u)), lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY))
    try:
        st, _ = lap.lap_solve(h, 1, 1, n, 1e-8)
        assert st == lap.LAP_EUNSUPPORTED
        assert lap.lap_apply_laplacian(h, 1, 1) == lap.LAP_EUNSUPPORTED
        assert lap.lap_apply_precond(h, 1, 1) == lap.LAP_EUNSUPPORTED
        st, _ = lap.lap_solve(h, 1, 1, n, -1.0)
        assert st == lap.LAP_EINVAL
    finally:
        lap.lap_free(h)


def test_default_params_and_status_strings():
    lap = _lap()
    p = lap.lap_default_params()
    assert p.mu == 0.8 and p.n_top == 2 and p.max_levels == 0 and p.max_iter == 1000
    assert lap.lap_status_str(lap.LAP_ENOCONV) == "LAP_ENOCONV"
    assert lap.lap_status_str(99) == "LAP_UNKNOWN"


def test_spectrum_and_mu_choice_errors_without_device():
    """The spectrum estimate and the choice of mu reject bad arguments and
    host-only hierarchies before touching a device."""
    import ctypes as C
    lap = _lap()
    n, u, v = W.grid2d(8)
    w = W.unit_weights(len(u))
    h = lap.lap_setup(n, u, v, w, lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY))
    try:
        b = np.ones(n)
        st, *_ = lap.lap_estimate_spectrum(h, b.ctypes.data, 10)
        assert st == lap.LAP_EUNSUPPORTED
        st, *_ = lap.lap_estimate_spectrum(h, b.ctypes.data, 0)
        assert st == lap.LAP_EINVAL
        st, *_ = lap.lap_estimate_spectrum(h, 0, 10)
        assert st == lap.LAP_EINVAL
    finally:
        lap.lap_free(h)
    st, best, _ = lap.lap_select_mu(n, u, v, w, [], 1, 10)
    assert st == lap.LAP_EINVAL and best == -1
    st, best, _ = lap.lap_select_mu(n, u, v, w, [0.8], 1, 0)
    assert st == lap.LAP_EINVAL
    # a mu outside (0, 1) fails in set-up for every candidate: its status
    kap = np.zeros(2)
    g, keep = lap._graph(n, u, v, w)
    p = lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY)
    mus = np.array([1.5, -0.2])
    bi = C.c_int32(-1)
    st = lap._lib.lap_select_mu(C.byref(g), C.byref(p), mus.ctypes.data, 2, C.c_void_p(1), 10,
                                kap.ctypes.data, C.byref(bi), None)
    assert st == lap.LAP_EINVAL and bi.value == -1
    assert np.all(np.isinf(kap))


@pytest.mark.parametrize("case", range(9))
def test_parallel_matching_hierarchy_bit_exact_vs_oracle(oracle_lib, case):
    """LAP_FLAG_PARALLEL_MATCHING on the host: the locally dominant rounds
    give the oracle's greedy matching (a global sort by edge weight), level
    by level, bit for bit, with the same coarse graphs."""
    from oracle import Graph, Hierarchy
    lap = _lap()
    name, (n, u, v), kind = _graphs()[case]
    w = _weights(kind, len(u), 100 + case)
    p = lap.lap_default_params(flags=lap.LAP_FLAG_HOST_ONLY | lap.LAP_FLAG_PARALLEL_MATCHING)
    h = lap.lap_setup(n, u, v, w, p)
    try:
        info = lap.lap_hierarchy_info(h)
        H = Hierarchy(Graph(n, u, v, w), matching="greedy")
        assert info["sizes"] == H.sizes, name
        for k in range(info["nlev"] - 1):
            a, m = lap.lap_export_level(h, k, info["sizes"][k])
            a2, m2 = H.agg(k)
            np.testing.assert_array_equal(a, a2)
            np.testing.assert_array_equal(m, m2)
        for k in range(info["nlev"]):
            pt, c, ww = lap.lap_export_graph(h, k, info["sizes"][k])
            pt2, c2, w2 = H.level_csr(k)
            np.testing.assert_array_equal(pt, pt2)
            np.testing.assert_array_equal(c, c2)
            np.testing.assert_array_equal(ww, w2)
    finally:
        lap.lap_free(h)
