"""Helpers for the GPU tests: torch device buffers around the C ABI."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


class GpuLap:
    """One hierarchy on cuda:0 (setup through lap_setup)."""

    def __init__(self, n, u, v, w, **params):
        import paper_2207_07847_amd as lap
        self.torch = torch_cuda()
        self.lap = lap
        self.n = int(n)
        p = lap.lap_default_params(**params)
        self.h = lap.lap_setup(n, u, v, w, p, self.stream())
        self.info = lap.lap_hierarchy_info(self.h)

    def stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def dev(self, a):
        return self.torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")

    def solve(self, b, tol):
        t = self.torch
        bd = self.dev(b)
        xd = t.full((self.n,), float("nan"), dtype=t.float64, device="cuda")
        st, info = self.lap.lap_solve(self.h, bd.data_ptr(), xd.data_ptr(), self.n, tol,
                                      stream=self.stream())
        t.cuda.synchronize()
        return st, xd.cpu().numpy(), info[0]

    def solve_many(self, B, tol, ld=None):
        """B: (nrhs, n) host array, column c = B[c]; returns (status, X, infos)."""
        t = self.torch
        nrhs = B.shape[0]
        ld = ld or self.n
        Bp = np.zeros((nrhs, ld))
        Bp[:, :self.n] = B
        bd = self.dev(Bp.ravel())
        xd = t.full((nrhs * ld,), float("nan"), dtype=t.float64, device="cuda")
        st, info = self.lap.lap_solve(self.h, bd.data_ptr(), xd.data_ptr(), self.n, tol,
                                      nrhs=nrhs, ld=ld, stream=self.stream())
        t.cuda.synchronize()
        return st, xd.cpu().numpy().reshape(nrhs, ld)[:, :self.n], info

    def apply_laplacian(self, x):
        xd = self.dev(x)
        yd = self.torch.empty_like(xd)
        st = self.lap.lap_apply_laplacian(self.h, xd.data_ptr(), yd.data_ptr(), self.stream())
        self.torch.cuda.synchronize()
        assert st == 0
        return yd.cpu().numpy()

    def apply_precond(self, r):
        rd = self.dev(r)
        zd = self.torch.empty_like(rd)
        st = self.lap.lap_apply_precond(self.h, rd.data_ptr(), zd.data_ptr(), self.stream())
        self.torch.cuda.synchronize()
        assert st == 0
        return zd.cpu().numpy()

    def estimate_spectrum(self, b, steps):
        bd = self.dev(b)
        out = self.lap.lap_estimate_spectrum(self.h, bd.data_ptr(), steps, self.stream())
        self.torch.cuda.synchronize()
        return out

    def close(self):
        if self.h:
            self.lap.lap_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
