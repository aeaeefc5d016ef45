"""lap_set_allocator: a hierarchy's device memory taken from the caller's
allocator (here torch's caching allocator), and released through it by
lap_free.  The solve on such a hierarchy is held to the same bars as the
parity tests (oracle iterate at the same count, true residual)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say, torch_cuda


def test_allocator_arguments():
    """Exactly one of the two functions NULL is an error (no device used)."""
    import paper_2207_07847_amd as lap
    assert lap.lap_set_allocator(alloc=lambda n: 0) == lap.LAP_EINVAL
    assert lap.lap_set_allocator(free=lambda p: None) == lap.LAP_EINVAL
    assert lap.lap_set_allocator() == lap.LAP_OK


@pytest.mark.gpu
def test_torch_allocator_holds_the_hierarchy(oracle_lib):
    import paper_2207_07847_amd as lap
    from oracle import MSP, Graph, Hierarchy, pcg
    torch = torch_cuda()
    n, u, v = W.grid3d(12, 10, 7)
    w = W.loguniform_weights(len(u), 31)
    b = W.gaussian_rhs(n, 32)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    assert lap.use_torch_allocator() == lap.LAP_OK
    try:
        G = GpuLap(n, u, v, w, mu=0.8, max_iter=5000)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - before
        dev = G.info["device_bytes"]
        try:
            st, x, info = G.solve(b, 1e-8)
        finally:
            G.close()
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated()
    finally:
        lap.lap_set_allocator()
    g = Graph(n, u, v, w)
    M = MSP(Hierarchy(g), 0.8)
    same = pcg(g, b, 0.0, info["iterations"], M)
    d = np.linalg.norm(x - same.x) / np.linalg.norm(same.x)
    msg = (f"hierarchy {dev} bytes, torch allocator holds {held} while set up, "
           f"{after - before} after lap_free; solve status {st}, {info['iterations']} "
           f"iterations, relres {info['relres_true']:.3e}, diff {d:.2e}")
    say(msg)
    assert dev > 0 and held >= dev, msg
    assert after == before, msg
    assert st == 0 and info["relres_true"] <= 1e-8 and d <= 1e-7, msg
    # later hierarchies use hipMalloc again: torch sees none of their memory
    G = GpuLap(n, u, v, w, mu=0.8)
    try:
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before, msg
    finally:
        G.close()
