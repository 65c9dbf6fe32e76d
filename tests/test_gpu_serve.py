"""Continuous batching on the GPU: requests of two volumes and two L5 values
arrive while others are iterating, join the running batches, and each
result equals the same request solved alone (the per-RHS arithmetic does not
depend on the batch it runs in, so the comparison is exact)."""
import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


def test_alone_equals_in_mix():
    import torch

    from paper_1810_01609_amd import mdwf as M
    from paper_1810_01609_amd.serve import GPUBackend, Request, percentiles, serve_gpu

    V1, V2 = (4, 4, 4, 8), (8, 4, 4, 8)
    be = GPUBackend([V1, V2], gauge_eps=0.2, inner="f32")
    try:
        reqs = [
            Request(0, 0.00, V1, 8, 0.05, 2, seed=100000),
            Request(1, 0.01, V1, 8, 0.02, 1, seed=100001),
            Request(2, 0.02, V2, 4, 0.05, 3, seed=100002),
            Request(3, 0.02, V1, 8, 0.03, 3, seed=100003),
            Request(4, 0.03, V2, 4, 0.04, 1, seed=100004),
            Request(5, 0.05, V1, 4, 0.05, 2, seed=100005),
        ]
        sched, sols, wall = serve_gpu(reqs, be, budget_bytes=8 << 30, iters_per_step=10, keep_solutions=True)
        log(f"[serve] wall {wall:.3f}s {percentiles(sched.done)}")
        assert len(sched.done) == len(reqs)
        assert sched.peak_used <= 8 << 30
        # some request was admitted while another of its lane was in flight
        by = {r.id: r for r in sched.done}
        assert by[1].t_admit < by[0].t_done or by[3].t_admit < by[1].t_done
        ctx = M.Context(0)
        for r in reqs:
            a = be.act(r)
            for k in range(r.nsrc):
                assert by[r.id].stats[k]["converged"] == 1
                eta = torch.zeros(a.spinor_shape(), dtype=torch.complex128, device="cuda")
                psi = torch.zeros_like(eta)
                ctx.source_z2(a, r.seed, k, eta)
                st = ctx.solve(be.gauge[tuple(r.volume)], a, be.opts(), eta, psi)[0]
                torch.cuda.synchronize()
                alone = psi.cpu().numpy()
                mixed = sols[r.id][k]
                assert st["iters"] == by[r.id].stats[k]["iters"]
                assert np.array_equal(alone, mixed), (r.id, k, np.abs(alone - mixed).max())
        ctx.close()
    finally:
        be.close()
