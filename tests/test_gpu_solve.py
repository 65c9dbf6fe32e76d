"""GPU propagator solves against the FP64 oracle.

The solve target is |b - A x| <= 1e-10 |b| on the normal equations; the
solution error against the oracle (solved to 1e-12) is held to 1e-8 relative,
and the FP64 full-5D residual |eta - D psi|/|eta| (recomputed here with the
oracle's D on the GPU's psi) to 1e-9.
"""
import numpy as np
import pytest

import mdwf_synth as S
import oracle as O
from gpu_util import empty_like_dev, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1810_01609_amd import mdwf as M

    c = M.Context(0)
    yield c
    c.close()


_cache = {}


def _c1(ctx):
    if "c1" not in _cache:
        U, act, oact = make_case((4, 4, 4, 8), 8, 0.05, 0.3, 1)
        g = ctx.gauge_load(act.lattice, U, precs=("f64", "f32", "f16", "bf16", "i16"))
        eta = O.point_source(oact, (0, 0, 0, 0), 0, 0)
        psi_o, info = O.solve(U, eta, oact, tol=1e-12)
        _cache["c1"] = (U, act, oact, g, eta, psi_o, info)
    return _cache["c1"]


@pytest.mark.parametrize("inner", ["f64", "f32", "f16", "bf16", "i16"])
def test_c1_solve_matches_oracle(ctx, inner):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, eta, psi_o, info = _c1(ctx)
    log(f"[solve] c1 inner={inner} oracle iters={info['iters']}")
    psi = empty_like_dev(eta.shape)
    st = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, inner=inner), to_dev(eta), psi)[0]
    log(f"   stats {st}")
    got = to_host(psi)
    assert st["status"] == M.OK and st["converged"] == 1
    assert st["rel_res_normal"] <= 1e-10
    err = rel(got, psi_o)
    assert err < 1e-8, err
    full = np.sqrt(O.norm2(eta - O.dirac(U, got, oact)) / O.norm2(eta))
    assert full < 1e-9, full
    assert abs(full - st["rel_res_full"]) < 1e-3 * full + 1e-14
    if inner != "f64":
        assert st["reliable_updates"] >= 2


def test_z2_solves_three_shapes(ctx):
    from paper_1810_01609_amd import mdwf as M

    for L, L5, mq, tap in [((6, 2, 2, 2), 3, 0.1, 1), ((8, 4, 4, 6), 5, 0.07, 0), ((4, 2, 2, 4), 1, 0.05, 1)]:
        U, act, oact = make_case(L, L5, mq, 0.3, 11, tap)
        g = ctx.gauge_load(L, U, precs=("f64", "f32"))
        eta = O.z2_source(oact, 77)
        psi_o, _ = O.solve(U, eta, oact, tol=1e-12)
        for inner in ("f64", "f32"):
            psi = empty_like_dev(eta.shape)
            st = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, inner=inner), to_dev(eta), psi)[0]
            log(f"[solve] {L} L5={L5} {inner}: {st['iters']} it, err={rel(to_host(psi), psi_o):.2e}")
            assert st["converged"] == 1
            assert rel(to_host(psi), psi_o) < 1e-8
        g.free()


def test_free_field_solution(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact = make_case((4, 4, 2, 4), 4, 0.1, 0.0, 0)
    g = ctx.gauge_load(act.lattice, U)
    eta = O.point_source(oact, (1, 2, 0, 3), 2, 1)
    psi = empty_like_dev(eta.shape)
    st = ctx.solve(g, act, M.CGOpts.make(tol=1e-12), to_dev(eta), psi)[0]
    assert st["converged"] == 1
    assert rel(to_host(psi), O.free_field_solve(eta, oact)) < 1e-9
    g.free()


def test_multi_rhs_equals_single_bitwise(ctx):
    """Each column of a fused multi-RHS solve is bitwise the single-RHS solve."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, *_ = _c1(ctx)
    n = 4
    etas = np.stack([O.point_source(oact, (0, 0, 0, 0), s, 1) for s in range(3)] + [O.z2_source(oact, 5)])
    for inner in ("f64", "f32", "f16", "i16"):
        opts = M.CGOpts.make(tol=1e-10, inner=inner)
        psi = empty_like_dev(etas.shape)
        stats = ctx.solve(g, act, opts, to_dev(etas), psi, nrhs=n)
        many = to_host(psi)
        for r in range(n):
            one = empty_like_dev(etas.shape[1:])
            s1 = ctx.solve(g, act, opts, to_dev(etas[r]), one)[0]
            assert s1["iters"] == stats[r]["iters"]
            assert np.array_equal(to_host(one), many[r]), (inner, r)


def test_determinism(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, eta, *_ = _c1(ctx)
    outs = []
    for _ in range(2):
        psi = empty_like_dev(eta.shape)
        ctx.solve(g, act, M.CGOpts.make(tol=1e-10, inner="f32"), to_dev(eta), psi)
        outs.append(to_host(psi))
    assert np.array_equal(outs[0], outs[1])


def test_initial_guess_resumes(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, eta, psi_o, _ = _c1(ctx)
    psi = to_dev(psi_o)
    st = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, use_initial_guess=1), to_dev(eta), psi)[0]
    assert st["converged"] == 1 and st["iters"] == 0
    # a half-converged guess finishes in fewer iterations than a cold start
    cold = ctx.solve(g, act, M.CGOpts.make(tol=1e-10), to_dev(eta), empty_like_dev(eta.shape))[0]
    part = empty_like_dev(eta.shape)
    ctx.solve(g, act, M.CGOpts.make(tol=1e-4), to_dev(eta), part)
    warm = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, use_initial_guess=1), to_dev(eta), part)[0]
    assert warm["converged"] == 1 and warm["iters"] < cold["iters"]
    assert rel(to_host(part), psi_o) < 1e-8


def test_failure_statuses(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, eta, *_ = _c1(ctx)
    psi = empty_like_dev(eta.shape)
    st = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, max_iter=3), to_dev(eta), psi, raise_on_fail=False)[0]
    assert st["status"] == M.ENOCONV and st["converged"] == 0 and st["iters"] == 3
    bad = eta.copy()
    bad[0, 0, 0, 0, 1, 2, 0] = np.nan
    st = ctx.solve(g, act, M.CGOpts.make(tol=1e-10), to_dev(bad), psi, raise_on_fail=False)[0]
    assert st["status"] == M.ENAN
    with pytest.raises(M.MDWFError) as e:
        ctx.solve(g, act, M.CGOpts.make(tol=-1.0), to_dev(eta), psi)
    assert e.value.status == M.EINVAL
    # zero source: psi = 0 at once
    st = ctx.solve(g, act, M.CGOpts.make(), to_dev(np.zeros_like(eta)), psi)[0]
    assert st["converged"] == 1 and st["iters"] == 0
    assert np.abs(to_host(psi)).max() == 0.0


def test_gauge_covariance_of_solution(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, eta, *_ = _c1(ctx)
    gt = S.random_gauge_transform(act.lattice, 3)
    gg = ctx.gauge_load(act.lattice, O.gauge_transform_links(U, gt), precs=("f64", "f32"))
    p1 = empty_like_dev(eta.shape)
    p2 = empty_like_dev(eta.shape)
    ctx.solve(g, act, M.CGOpts.make(tol=1e-12, inner="f32"), to_dev(eta), p1)
    ctx.solve(gg, act, M.CGOpts.make(tol=1e-12, inner="f32"), to_dev(O.gauge_transform_spinor(eta, gt)), p2)
    assert rel(to_host(p2), O.gauge_transform_spinor(to_host(p1), gt)) < 1e-9
    gg.free()


@pytest.mark.parametrize("sample", [1, 7])
def test_profile_counts_working_launches(ctx, sample):
    """Kernel-time accounting: the inner stencil class counts the four
    launches of every iteration that did work (launches issued after the
    solve froze itself waiting for the host are left out) plus the M_phi p
    launches of the setup and of the reliable updates."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, eta, *_ = _c1(ctx)
    psi = empty_like_dev(eta.shape)
    ctx.profile_enable(True, sample=sample)
    ctx.profile_reset()
    st = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, inner="f32"), to_dev(eta), psi)[0]
    d = ctx.profile_read(M.PROF_DSLASH_INNER)
    ctx.profile_enable(False)
    lo = 4 * st["iters"] + 1
    assert lo <= d["launches"] <= lo + st["reliable_updates"], (d, st)
    assert d["ms"] > 0 and d["bytes"] > 0


def test_graph_replay_equals_eager(ctx, monkeypatch):
    """The CG iteration captured once into a HIP graph and replayed (between
    the replays: the host's polls, reliable updates in FP64, the batch
    shrinking when a RHS converges and the graph being captured again) gives
    bitwise the solutions and iteration counts of the launches issued one by
    one, for two jobs of different masses stepped together."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, *_ = _c1(ctx)
    acts = [M.Action.make(act.lattice, act.L5, 1.5, 0.5, 1.3, mq) for mq in (0.05, 0.1)]
    etas = [np.stack([O.z2_source(oact, 40 + r, rhs=r) for r in range(2)]), O.point_source(oact, (1, 0, 0, 1), 2, 0)[None]]
    outs = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("MDWF_GRAPH", mode)
        for inner in ("f32", "f16"):
            opts = M.CGOpts.make(tol=1e-10, inner=inner)
            psis = [empty_like_dev(e.shape) for e in etas]
            jobs = [ctx.job_begin(g, a, opts, to_dev(e), p, nrhs=e.shape[0]) for a, e, p in zip(acts, etas, psis)]
            while not all(j.poll()[0] for j in jobs):
                assert ctx.job_step(jobs, 1000) == M.OK
            stats = [j.poll()[1] for j in jobs]
            for j in jobs:
                j.end()
            outs[(mode, inner)] = ([to_host(p) for p in psis], [[s["iters"] for s in st] for st in stats])
            log(f"[graph] MDWF_GRAPH={mode} {inner}: iterations {outs[(mode, inner)][1]}")
    for inner in ("f32", "f16"):
        (pa, ia), (pb, ib) = outs[("0", inner)], outs[("1", inner)]
        assert ia == ib
        for x, y in zip(pa, pb):
            assert np.array_equal(x, y)
    # and the solutions are right
    psi_o, _ = O.solve(U, etas[1][0], O.Action(act.lattice, act.L5, 1.5, 0.5, 1.3, 0.1), tol=1e-12)
    assert rel(outs[("1", "f32")][0][1][0], psi_o) < 1e-8


def test_many_reliable_updates(ctx):
    """delta = 0.9 forces a reliable update nearly every iteration: four fused
    RHS make several hundred updates in one step call, so the small-table
    region the updates upload through wraps around several times while the
    CG loop keeps reading its own tables from it; every solution still
    matches the oracle's."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, *_ = _c1(ctx)
    etas = np.stack([O.z2_source(oact, 60 + r, rhs=r) for r in range(4)])
    psi = empty_like_dev(etas.shape)
    stats = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, inner="f32", delta=0.9), to_dev(etas), psi, nrhs=4)
    got = to_host(psi)
    total = sum(s["reliable_updates"] for s in stats)
    log(f"[solve] delta 0.9: {total} reliable updates, iterations {[s['iters'] for s in stats]}")
    assert total > 150
    for r in range(4):
        assert stats[r]["converged"] == 1
        psi_o, _ = O.solve(U, etas[r], oact, tol=1e-12)
        assert rel(got[r], psi_o) < 1e-8


@pytest.mark.parametrize("inner", ["f64", "f32", "f16"])
def test_x_update_placement_is_bitwise_neutral(ctx, monkeypatch, inner):
    """The CG's x += alpha p runs in the second M^+ launch (with r -= alpha q)
    or in the first one (MDWF_X_IN_B1); both apply the same alpha to the same
    p, so solutions, iteration counts and reliable updates agree bitwise, for
    three fused RHS of a z2 source stepped through several updates."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, *_ = _c1(ctx)
    eta = np.stack([O.z2_source(oact, 70 + r, rhs=r) for r in range(3)])
    outs = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("MDWF_X_IN_B1", mode)
        psi = empty_like_dev(eta.shape)
        st = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, inner=inner), to_dev(eta), psi, nrhs=3)
        outs[mode] = (to_host(psi), [(s["iters"], s["reliable_updates"]) for s in st])
        log(f"[x-update] MDWF_X_IN_B1={mode} {inner}: {outs[mode][1]}")
    assert outs["0"][1] == outs["1"][1]
    assert np.array_equal(outs["0"][0], outs["1"][0])
    psi_o, _ = O.solve(U, eta[2], oact, tol=1e-12)
    assert rel(outs["1"][0][2], psi_o) < 1e-8
