"""Named small parity workloads shared by the GPU parity tests and the script
that stores their oracle iteration bands (tests/golden/make_iteration_bands.py).
Each is (n, u, v, w, mu, rhs) from the seeded generators of ``workloads``."""
import numpy as np

import workloads as W


def case(name):
    """(n, u, v, w, mu, rhs) for a named small workload."""
    if name == "grid2d_64_lowfreq":
        n, u, v = W.grid2d(64)
        return n, u, v, W.unit_weights(len(u)), 0.8, W.lowfreq_rhs(n)
    if name == "grid3d_16_loguniform":
        n, u, v, w = W.config_graph("grid3d_128", 16 / 128)
        return n, u, v, w, 0.8, W.gaussian_rhs(n, W.MASTER_SEED + 3)
    if name == "grid3d_12x10x7_loguniform":
        n, u, v = W.grid3d(12, 10, 7)
        return n, u, v, W.loguniform_weights(len(u), 31), 0.8, W.gaussian_rhs(n, 32)
    if name == "er_3000_uniform":
        n, u, v = W.erdos_renyi(3000, 6, 7)
        return n, u, v, W.uniform01_weights(len(u), 8), 0.8, W.gaussian_rhs(n, 9)
    if name == "chunglu_6000":
        n, u, v = W.chung_lu(6000, 16.0, 2.1, 10)
        return n, u, v, W.uniform01_weights(len(u), 11), 0.8, W.gaussian_rhs(n, 12)
    if name == "ring_1024":
        n, u, v = W.ring(1024)
        return n, u, v, W.unit_weights(len(u)), 0.8, W.lowfreq_rhs(n)
    if name == "ring_1024_quarter":
        # mu = n^(-1/4), the setting that fits Table 2's rings
        n, u, v = W.ring(1024)
        return n, u, v, W.unit_weights(len(u)), 1024 ** -0.25, W.lowfreq_rhs(n)
    if name == "ring_1024_mu03":
        n, u, v = W.ring(1024)
        return n, u, v, W.unit_weights(len(u)), 0.3, W.lowfreq_rhs(n)
    if name == "grid3d_12_quarter":
        # mu = n^(-1/4) on a weighted 3D grid: PCG does not converge with the
        # MSP at this mu, so it is a preconditioner case only
        n, u, v = W.grid3d(12, 12, 12)
        return n, u, v, W.loguniform_weights(len(u), 31), n ** -0.25, W.gaussian_rhs(n, 32)
    if name == "grid2d_32_invsqrt":
        # mu = 1/sqrt(n), the setting of Tables 2-3 (a preconditioner case)
        n, u, v = W.grid2d(32)
        return n, u, v, W.unit_weights(len(u)), n ** -0.5, W.gaussian_rhs(n, 33)
    if name == "grid2d_64_mu05":
        n, u, v = W.grid2d(64)
        return n, u, v, W.unit_weights(len(u)), 0.5, W.gaussian_rhs(n, 17)
    if name == "ws_2000":
        n, u, v = W.watts_strogatz(2000, 4, 2000 ** -0.5, 13)
        return n, u, v, W.unit_weights(len(u)), 0.8, W.gaussian_rhs(n, 14)
    if name == "path_3":
        n, u, v = W.path(3)
        return n, u, v, np.array([1.0, 2.0]), 0.8, np.array([1.0, 0.0, -1.0])
    if name == "path_2":
        return 2, np.array([0]), np.array([1]), np.array([3.0]), 0.8, np.array([1.0, -1.0])
    if name == "star_61":
        # a star cannot be coarsened: one level, solved exactly on chip
        n, u, v = 61, np.zeros(60, dtype=np.int64), np.arange(1, 61)
        return n, u, v, W.uniform01_weights(60, 15), 0.5, W.gaussian_rhs(n, 16)
    raise KeyError(name)


PCG_CASES = ["grid2d_64_lowfreq", "grid3d_16_loguniform", "grid3d_12x10x7_loguniform",
             "er_3000_uniform", "chunglu_6000", "ring_1024", "grid2d_64_mu05", "ws_2000",
             "path_3", "path_2", "star_61", "ring_1024_quarter", "ring_1024_mu03"]

# Below this mu the oracle's elimination of T~ in the expanded space is no
# longer accurate to FP64 rounding (tests/test_oracle_closed.py), so the
# bands and references of those cases use the closed form alone.
ELIM_MIN_MU = 0.5


def plain_cg_case():
    """Unpreconditioned CG (LAP_PREC_NONE) on a weighted 32 x 20 grid."""
    n, u, v = W.grid2d(32, 20)
    return n, u, v, W.uniform01_weights(len(u), 3), None, W.gaussian_rhs(n, 4)


def hub_case():
    """Chung-Lu graph plus a hub with 6000 neighbours and 3000 pendants."""
    n, u, v = W.hub_graph(20000, 6000, 3000, 7)
    return n, u, v, W.uniform01_weights(len(u), 71), 0.8, W.gaussian_rhs(n, 72)
