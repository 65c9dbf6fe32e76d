"""The launch autotuner: it searches the sites-per-workgroup of the fused
stencil per key, keeps the result in its table (save / load round trip), and
never changes a result: tuned and untuned runs are bitwise equal."""
import numpy as np
import pytest

import mdwf_synth as S
from gpu_util import empty_like_dev, make_case, to_dev, to_host

pytestmark = pytest.mark.gpu


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
    for p in ("f64", "f32", "f16"):
        assert np.array_equal(outs[(0, p)], outs[(1, p)]), p
    assert outs[(0, "solve")][1] == outs[(1, "solve")][1]
    assert np.array_equal(outs[(0, "solve")][0], outs[(1, "solve")][0])
