"""The launch autotuner: it searches the sites per workgroup and the
traversal of the fused stencil per key and keeps the result in its table
(save / load round trip).  Every candidate it can choose is run on its own
(MDWF_CB_LOG2, MDWF_BT, MDWF_YB, MDWF_RHS_ORDER) and checked against the FP64 oracle's
M^+M^ at the precision's bar and against the default launch bitwise (the
candidates only change which workgroup computes which sites, never the
per-site arithmetic), and tuned runs equal untuned runs bitwise."""
import numpy as np
import pytest

import mdwf_synth as S
import oracle as O
from gpu_util import check, empty_like_dev, log, make_case, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 8e-3}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_every_candidate_matches_oracle(prec, monkeypatch):
    from paper_1810_01609_amd import mdwf as M

    # 32 x 8 sites per xy-plane of one parity (256): whole workgroups of 16-128
    # sites; Lt = 8 admits Bt = 2, 4, 8; Ly = 16 admits 4-row bands
    U, act, oact = make_case((32, 16, 2, 8), 4, 0.03, 0.2, 12)
    ctx = M.Context(0)
    g = ctx.gauge_load(act.lattice, U, precs=("f64", prec))
    # three RHS: every RHS order (side by side, RHS by RHS, RHS by RHS per XCD
    # eighth) takes the slots through a different workgroup mapping
    x = S.random_spinor(act.lattice, act.L5, 21, nrhs=3)
    Me = O.parity_mask(oact, 0)
    want = [O.normal_op(U, Me * x[r], oact) for r in range(3)]
    ref = None
    cands = [(lg, bt, yb, o) for lg in (4, 5, 6, 7) for bt, yb in ((0, 1), (2, 1), (4, 1), (8, 1), (2, 4), (4, 4))
             for o in (0, 1, 2)]
    for lg, bt, yb, o in cands:
        monkeypatch.setenv("MDWF_CB_LOG2", str(lg))
        monkeypatch.setenv("MDWF_BT", str(bt))
        monkeypatch.setenv("MDWF_YB", str(yb))
        monkeypatch.setenv("MDWF_RHS_ORDER", str(o))
        out = empty_like_dev(x.shape)
        ctx.dslash(g, act, M.OP_NORMAL, prec, to_dev(x), out, nrhs=3)
        got = to_host(out)
        for r in range(3):
            check(got[r], want[r], TOL[prec], f"{prec} {1 << lg} sites/workgroup Bt={bt} bands={yb} order {o} rhs {r}")
        if ref is None:
            ref = got
        assert np.array_equal(got, ref), (lg, bt, yb, o)
    g.free()
    ctx.close()


def test_tuned_equals_untuned(tmp_path):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact = make_case((8, 8, 8, 8), 12, 0.02, 0.2, 3)
    x = S.random_spinor(act.lattice, act.L5, 1, nrhs=2)
    outs = {}
    for mode in (0, 1):
        ctx = M.Context(0)
        ctx.tune_mode(mode)
        g = ctx.gauge_load(act.lattice, U, precs=("f64", "f32", "f16"))
        for p in ("f64", "f32", "f16"):
            out = empty_like_dev(x.shape)
            ctx.dslash(g, act, M.OP_NORMAL, p, to_dev(x), out, nrhs=2)
            outs[(mode, p)] = to_host(out)
        eta = to_dev(x[0])
        psi = empty_like_dev(x.shape[1:])
        st = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, inner="f32"), eta, psi)[0]
        outs[(mode, "solve")] = (to_host(psi), st["iters"])
        if mode == 1:
            n = ctx.tune_entries()
            assert n >= 3
            path = tmp_path / "tune.txt"
            ctx.tune_save(path)
            lines = open(path).read().strip().splitlines()
            assert len(lines) == n and all(" | " in l for l in lines)
            c2 = M.Context(0)
            c2.tune_load(path)
            assert c2.tune_entries() == n
            c2.close()
        g.free()
        ctx.close()
    Me = O.parity_mask(oact, 0)
    for p in ("f64", "f32", "f16"):
        assert np.array_equal(outs[(0, p)], outs[(1, p)]), p
        check(outs[(1, p)][0], O.normal_op(U, Me * x[0], oact), TOL[p], f"tuned M^+M^ {p}")
    assert outs[(0, "solve")][1] == outs[(1, "solve")][1]
    assert np.array_equal(outs[(0, "solve")][0], outs[(1, "solve")][0])
