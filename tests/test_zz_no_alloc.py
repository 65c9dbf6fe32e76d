"""mdwf_dslash_noalloc against mdwf_dslash: the same kernels on the same
inputs, so the fields are bitwise equal; two calls in a row, the second on a
smaller input, and the device's free memory unchanged across a call.  Sizes
beyond the scratch's limits are rejected."""
import numpy as np
import pytest

import mdwf_synth as S
import oracle as O
from gpu_util import check, empty_like_dev, log, make_case, to_dev, to_host

pytestmark = pytest.mark.gpu

# (lattice, L5, precision, operator, right-hand sides): the second is smaller
CASES = [((8, 4, 4, 8), 8, "f32", "NORMAL", 3), ((4, 4, 2, 4), 4, "f16", "D", 1)]


def test_noalloc_equals_dslash_twice():
    import torch

    from paper_1810_01609_amd import mdwf as M

    ctx = M.Context(0)
    for (L, L5, prec, op, nrhs) in CASES:
        log(f"[noalloc] {L} L5={L5} {prec} {op} nrhs={nrhs}")
        U, act, oact = make_case(L, L5, 0.05, 0.3, 3)
        g = ctx.gauge_load(L, U, precs=("f64", prec))
        x = S.random_spinor(L, L5, 5, nrhs=nrhs)
        xd = to_dev(x)
        ref = empty_like_dev(x.shape)
        got = empty_like_dev(x.shape)
        ctx.dslash(g, act, getattr(M, "OP_" + op), prec, xd, ref, nrhs=nrhs)
        ctx.dslash_noalloc(g, act, getattr(M, "OP_" + op), prec, xd, got, nrhs=nrhs)
        r, o = to_host(ref), to_host(got)
        assert np.array_equal(r, o)
        Me = O.parity_mask(oact, 0)
        for k in range(nrhs):
            want = O.normal_op(U, Me * x[k], oact) if op == "NORMAL" else O.dirac(U, x[k], oact)
            check(o[k], want, 1e-6 if prec == "f32" else 8e-3, f"noalloc {op} {prec} rhs {k} vs oracle")
        # no allocation: the device's free memory is the same before and after
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ctx.dslash_noalloc(g, act, getattr(M, "OP_" + op), prec, xd, got, nrhs=nrhs)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert np.array_equal(to_host(got), r)
        g.free()
    ctx.close()


def test_noalloc_rejects_beyond_its_scratch():
    from paper_1810_01609_amd import mdwf as M

    ctx = M.Context(0)
    L, L5 = (4, 4, 4, 8), 8
    U, act, oact = make_case(L, L5, 0.05, 0.3, 3)
    g = ctx.gauge_load(L, U, precs=("f64",))
    x = empty_like_dev((17,) + act.spinor_shape())
    y = empty_like_dev((17,) + act.spinor_shape())
    with pytest.raises(M.MDWFError, match="exceeds the maximum"):
        ctx.dslash_noalloc(g, act, M.OP_D, "f64", x, y, nrhs=17)
    g.free()
    big = M.Action.make((16, 16, 16, 32), 12, mq=0.02)  # FP64: 5 half-fields of 151 MB
    Ub = S.gauge_field(big.lattice, 0.2, 2)
    gb = ctx.gauge_load(big.lattice, Ub, precs=("f64",))
    xb = empty_like_dev(big.spinor_shape())
    yb = empty_like_dev(big.spinor_shape())
    with pytest.raises(M.MDWFError, match="bytes of scratch"):
        ctx.dslash_noalloc(gb, big, M.OP_D, "f64", xb, yb)
    gb.free()
    ctx.close()
