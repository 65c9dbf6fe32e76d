"""The hop computed as one rank of a 4D domain-decomposed run computes it
(face packing, interior hop without the hops across split boundaries,
exterior update from the packed faces), with the lattice as its own neighbour
in every split dimension: it must reproduce H_eo of the FP64 oracle to the
precision's tolerance, and the plain fused hop to rounding (the hops across
split boundaries are summed after the others)."""
import numpy as np
import pytest

import mdwf_synth as S
import oracle as O
from gpu_util import check, empty_like_dev, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 8e-3, "bf16": 6e-2, "i16": 1e-3}
# against the unsplit GPU hop in the same precision: reordered sums (FP64,
# FP32) or one more rounding of the stored result (16-bit storage)
TOL_SAME = {"f64": 1e-15, "f32": 5e-7, "f16": 4e-3, "bf16": 3e-2, "i16": 5e-4}

CASES = {
    "c1": ((4, 4, 4, 8), 8, 0.05, 0.3, 1, 1),
    "tiles": ((8, 4, 4, 6), 5, 0.07, 0.3, 6, 0),
    "aniso_l5_16": ((10, 4, 2, 6), 16, 0.02, 0.2, 8, 1),
    "ragged": ((6, 2, 2, 2), 3, 0.1, 0.3, 5, 1),
}
MASKS = [1, 2, 4, 8, 6, 14, 15]


@pytest.fixture(scope="module")
def ctx():
    from paper_1810_01609_amd import mdwf as M

    c = M.Context(0)
    yield c
    c.close()


_cache = {}


def _setup(ctx, name):
    if name not in _cache:
        L, L5, mq, eps, seed, tap = CASES[name]
        U, act, oact = make_case(L, L5, mq, eps, seed, tap)
        g = ctx.gauge_load(L, U, precs=("f64", "f32", "f16", "bf16", "i16"))
        x = S.random_spinor(L, L5, 500 + seed)
        _cache[name] = (U, act, oact, g, x, O.hop_eo(U, x, oact))
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16", "i16"])
def test_split_hop_matches(ctx, name, prec):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, x, expect = _setup(ctx, name)
    xd = to_dev(x)
    ref = empty_like_dev(x.shape)
    ctx.dslash(g, act, M.OP_HOP_EO, prec, xd, ref)
    ref_h = to_host(ref)
    out = empty_like_dev(x.shape)
    ctx.hop_split(g, act, prec, 0, xd, out)
    assert np.array_equal(to_host(out), ref_h), "split_mask 0 is the plain hop"
    for mask in MASKS:
        log(f"[split] {name} {prec} mask={mask:04b}")
        out = empty_like_dev(x.shape)
        ctx.hop_split(g, act, prec, mask, xd, out)
        got = to_host(out)
        assert np.abs(O.parity_mask(oact, 1) * got).max() == 0.0
        check(got, expect, TOL[prec], f"split {name} {prec} mask {mask:04b} vs oracle")
        check(got, ref_h, TOL_SAME[prec], f"split {name} {prec} mask {mask:04b} vs unsplit")


def test_split_hop_benchmark_block(ctx):
    """The block the benchmark times (one rank of c4 split 2x2x2 in y, z, t:
    32x16x16x32, L5 = 12, y-band traversal): split against unsplit hop."""
    import torch

    from paper_1810_01609_amd import mdwf as M

    c = S.CONFIGS["c4"]
    L = (32, 16, 16, 32)
    act = M.Action.make(L, c["L5"], c["b5"], c["c5"], c["M5"], c["mq"])
    g = ctx.gauge_load(L, S.gauge_field(L, c["eps"], c["seed"]), precs=("f64", "f32", "f16"))
    x = torch.zeros(act.spinor_shape(), dtype=torch.complex128, device="cuda")
    ctx.source_z2(act, 7, 0, x)
    ref = torch.zeros_like(x)
    out = torch.zeros_like(x)
    for prec in ("f64", "f32", "f16"):
        log(f"[split] benchmark block {prec}")
        ctx.dslash(g, act, M.OP_HOP_EO, prec, x, ref)
        ctx.hop_split(g, act, prec, 0b1110, x, out)
        err = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
        assert err < TOL_SAME[prec], (prec, err)
    del x, ref, out
    g.free()


def test_split_hop_multi_rhs_and_timing(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, *_ = _setup(ctx, "tiles")
    n = 3
    x = S.random_spinor(act.lattice, act.L5, 600, nrhs=n)
    xd = to_dev(x)
    out = empty_like_dev(x.shape)
    ms = ctx.hop_split(g, act, "f32", 14, xd, out, nrhs=n, timed=True)
    assert len(ms) == 3 and all(t >= 0.0 for t in ms)
    got = to_host(out)
    for r in range(n):
        one = empty_like_dev(x.shape[1:])
        ctx.hop_split(g, act, "f32", 14, to_dev(x[r]), one)
        assert np.array_equal(to_host(one), got[r])
        assert rel(got[r], O.hop_eo(U, x[r], oact)) < TOL["f32"]


def test_split_hop_rejects(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g, x, _ = _setup(ctx, "c1")
    xd = to_dev(x)
    out = empty_like_dev(x.shape)
    for mask in (-1, 16):
        with pytest.raises(M.MDWFError):
            ctx.hop_split(g, act, "f32", mask, xd, out)
    # extents are checked before anything else: Ly = 3 is odd, and the x
    # faces need an even Ly
    odd = M.Action.make((4, 3, 4, 8), act.L5, 1.5, 0.5, 1.3, 0.05)
    xo = empty_like_dev(odd.spinor_shape())
    oo = empty_like_dev(odd.spinor_shape())
    for mask in (1, 2):
        with pytest.raises(M.MDWFError, match="even"):
            ctx.hop_split(g, odd, "f32", mask, xo, oo)
    # a gauge field of another lattice
    with pytest.raises(M.MDWFError, match="differs"):
        ctx.hop_split(g, odd, "f32", 12, xo, oo)
