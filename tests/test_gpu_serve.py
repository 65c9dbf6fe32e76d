"""Continuous batching on the GPU: requests of two volumes and two L5 values
arrive while others are iterating, join the running batches (one fused batch
mixes three quark masses), and every served result is checked twice: it
equals the same request solved alone (the per-RHS arithmetic does not depend
on the batch it runs in, so the comparison is exact) and it matches the FP64
oracle's solution (solved to 1e-12) to the 1e-8 solution bar.  The plain
FP64 first-in-first-out baseline is checked against the oracle the same way."""
import numpy as np
import pytest

import mdwf_synth as S
import oracle as O
from gpu_util import log, rel

pytestmark = pytest.mark.gpu

V1, V2 = (4, 4, 4, 8), (8, 4, 4, 8)


def _reqs():
    from paper_1810_01609_amd.serve import Request

    return [
        Request(0, 0.00, V1, 8, 0.05, 2, seed=100000),
        Request(1, 0.01, V1, 8, 0.02, 1, seed=100001),
        Request(2, 0.02, V2, 4, 0.05, 3, seed=100002),
        Request(3, 0.02, V1, 8, 0.03, 3, seed=100003),
        Request(4, 0.03, V2, 4, 0.04, 1, seed=100004),
        Request(5, 0.05, V1, 4, 0.05, 2, seed=100005),
    ]


_oracle_cache = {}


def _oracle_solution(r, k):
    """The oracle's solution for source k of request r (gauge fields as the
    backend draws them: eps 0.2, seeds 11, 12 for V1, V2)."""
    key = (r.id, k)
    if key not in _oracle_cache:
        U = S.gauge_field(r.volume, 0.2, 11 if tuple(r.volume) == V1 else 12)
        oact = O.Action(r.volume, r.L5, 1.5, 0.5, 1.3, r.mq)
        psi, _ = O.solve(U, O.z2_source(oact, r.seed, rhs=r.src_offset + k), oact, tol=1e-12)
        _oracle_cache[key] = psi
    return _oracle_cache[key]


def test_alone_equals_in_mix_and_oracle():
    import torch

    from paper_1810_01609_amd import mdwf as M
    from paper_1810_01609_amd.serve import GPUBackend, percentiles, serve_gpu

    be = GPUBackend([V1, V2], gauge_eps=0.2, inner="f32")
    try:
        reqs = _reqs()
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
                err = rel(mixed, _oracle_solution(r, k))
                log(f"   request {r.id} (V={r.volume} L5={r.L5} mq={r.mq}) source {k}: "
                    f"{st['iters']} it, error vs oracle {err:.2e}")
                assert err < 1e-8, (r.id, k, err)
        ctx.close()
    finally:
        be.close()


def test_fifo_fp64_baseline_matches_oracle():
    from paper_1810_01609_amd.serve import GPUBackend, percentiles, serve_fifo

    be = GPUBackend([V1, V2], gauge_eps=0.2, inner="f64")
    try:
        reqs = _reqs()[:3]
        done, sols, wall = serve_fifo(reqs, be, keep_solutions=True)
        log(f"[fifo] wall {wall:.3f}s {percentiles(done)}")
        assert [r.id for r in done] == [0, 1, 2]
        assert all(done[i].t_admit >= done[i - 1].t_done for i in range(1, len(done)))  # one at a time
        for r in done:
            for k in range(r.nsrc):
                assert r.stats[k]["converged"] == 1
                err = rel(sols[r.id][k], _oracle_solution(r, k))
                assert err < 1e-8, (r.id, k, err)
    finally:
        be.close()


def test_ended_job_releases_its_tensors():
    """A job keeps its source and solution tensors alive while it runs and
    lets go of them when it ends, even while the Job object itself is still
    referenced (a serving lane keeps its last batch of jobs in a list): the
    device memory torch holds for them is freed at end(), not later."""
    import torch

    from paper_1810_01609_amd import mdwf as M

    L, L5 = (8, 8, 8, 16), 8
    act = M.Action.make(L, L5, 1.5, 0.5, 1.3, 0.05)
    ctx = M.Context(0)
    g = ctx.gauge_load(L, S.gauge_field(L, 0.2, 5), precs=("f64", "f16"))
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    eta = torch.zeros((2,) + act.spinor_shape(), dtype=torch.complex128, device="cuda")
    psi = torch.zeros_like(eta)
    nbytes = 2 * eta.numel() * eta.element_size()
    for k in range(2):
        ctx.source_z2(act, 9, k, eta[k])
    job = ctx.job_begin(g, act, M.CGOpts.make(tol=1e-10, inner="f16"), eta, psi, nrhs=2)
    del eta, psi
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base >= nbytes  # held by the running job
    while not job.poll()[0]:
        assert ctx.job_step([job], 200) == M.OK
    job.end()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base < nbytes, "the ended job still holds its tensors"
    assert job is not None
    g.free()
    ctx.close()
