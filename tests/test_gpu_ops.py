"""GPU parity of every operator of the C ABI against the FP64 CPU oracle.

Element-wise comparison on seeded inputs at sizes the oracle finishes in
seconds, covering several workgroup tiles, ragged tails (sites per parity not
a multiple of 16/32/64), L5 = 1, a large L5, periodic and antiperiodic time,
the free field, and all four storage precisions.

Every comparison checks the norm-wise relative error |got - ref| / |ref| and
the element-wise one max|got - ref| / max|ref| against the same bar, and logs
both.  Bars:

* FP64 1e-13: ~1e3 flops per output, each rounded at 2^-53 ~ 1.1e-16.
* FP32 1e-6 (the dslash bar FP32 results are held to): the input is rounded
  to FP32 once (2^-24 ~ 6e-8 relative) and each launch sums ~100 terms per
  output in FP32; the deepest operator (M^+M^, four launches) stays below
  ~1e-6.
* 16-bit storage with one FP32 scale per 5D site: the storage unit roundoff u
  is 2^-11 (FP16), 2^-8 (BF16), 1/(2*32767) (int16 of the site maximum).
  Every stored field (the input and the output of each launch, up to five for
  M^+M^) adds an error of at most u times the site maximum; the operators
  between them have norm <= ~2 and the errors add in norm, so the bar is
  16u: FP16 8e-3, BF16 6e-2, int16 1e-3 (the int16 bar 16u = 2.4e-4 is
  raised to 1e-3 because the stored integers enter FP32 arithmetic unscaled
  and sites far below their neighbours lose relative precision).
"""
import numpy as np
import pytest

import mdwf_synth as S
import oracle as O
from gpu_util import check, empty_like_dev, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 8e-3, "bf16": 6e-2, "i16": 1e-3}

CASES = {
    # name: (L, L5, mq, eps, seed, t_antiperiodic)
    "c1": ((4, 4, 4, 8), 8, 0.05, 0.3, 1, 1),
    "ragged": ((6, 2, 2, 2), 3, 0.1, 0.3, 5, 1),
    "tiles": ((8, 4, 4, 6), 5, 0.07, 0.3, 6, 0),
    "l5one": ((4, 2, 2, 4), 1, 0.05, 0.3, 7, 1),
    "aniso_l5_16": ((10, 4, 2, 6), 16, 0.02, 0.2, 8, 1),
    "free": ((4, 4, 2, 4), 4, 0.1, 0.0, 0, 1),
    # xy-plane of 64 sites per parity: the blocked (z, t) traversal engages
    "blocked": ((16, 8, 4, 8), 4, 0.05, 0.3, 9, 1),
    # xy-plane of 512 sites per parity: the traversal also cuts it into y-bands
    "banded": ((32, 32, 2, 4), 2, 0.05, 0.3, 10, 1),
}


def _oracle(op, U, x, a):
    Me = O.parity_mask(a, 0)
    Mo = O.parity_mask(a, 1)
    return {
        "D": lambda: O.dirac(U, x, a),
        "DDAG": lambda: O.dirac_dag(U, x, a),
        "MHAT": lambda: O.mhat(U, Me * x, a),
        "MHATDAG": lambda: O.mhat_dag(U, Me * x, a),
        "NORMAL": lambda: O.normal_op(U, Me * x, a),
        "HOP_EO": lambda: O.hop_eo(U, x, a),
        "HOP_OE": lambda: O.hop_oe(U, x, a),
        "HOP": lambda: O.hop(U, x, a),
        "HOPDAG": lambda: O.hop_dag(U, x, a),
        "M5": lambda: O.m5(x, a),
        "M5INV": lambda: O.m5_inv(x, a),
        "MPHI": lambda: O.m_phi(x, a),
        "PREP": lambda: Me * O.prep_source(U, x, a),
    }[op]()


OPS = ["D", "DDAG", "MHAT", "MHATDAG", "NORMAL", "HOP_EO", "HOP_OE", "HOP", "HOPDAG", "M5", "M5INV", "MPHI", "PREP"]


@pytest.fixture(scope="module")
def ctx():
    from paper_1810_01609_amd import mdwf as M

    c = M.Context(0)
    yield c
    c.close()


_gauges = {}


def _setup(ctx, name):
    L, L5, mq, eps, seed, tap = CASES[name]
    U, act, oact = make_case(L, L5, mq, eps, seed, tap)
    if name not in _gauges:
        _gauges[name] = ctx.gauge_load(L, U, precs=("f64", "f32", "f16", "bf16", "i16"))
    return U, act, oact, _gauges[name]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("op", OPS)
def test_op_f64(ctx, name, op):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, name)
    log(f"[op] {name} {op} f64 L={act.lattice} L5={act.L5}")
    x = S.random_spinor(act.lattice, act.L5, 100 + OPS.index(op))
    expect = _oracle(op, U, x, oact)
    xi = to_dev(x)
    out = empty_like_dev(x.shape)
    ctx.dslash(g, act, getattr(M, "OP_" + op), "f64", xi, out)
    got = to_host(out)
    check(got, expect, TOL["f64"], f"{name} {op} f64")
    # untouched parity of half-field outputs is exactly zero
    if op in ("MHAT", "MHATDAG", "NORMAL", "HOP_EO", "PREP"):
        assert np.abs(O.parity_mask(oact, 1) * got).max() == 0.0
    if op == "HOP_OE":
        assert np.abs(O.parity_mask(oact, 0) * got).max() == 0.0


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16", "i16"])
@pytest.mark.parametrize("name", ["c1", "ragged", "aniso_l5_16"])
@pytest.mark.parametrize("op", ["D", "NORMAL", "HOP", "M5INV", "PREP", "MHATDAG"])
def test_op_low_precision(ctx, prec, name, op):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, name)
    log(f"[op] {name} {op} {prec}")
    x = S.random_spinor(act.lattice, act.L5, 200 + OPS.index(op))
    expect = _oracle(op, U, x, oact)
    out = empty_like_dev(x.shape)
    ctx.dslash(g, act, getattr(M, "OP_" + op), prec, to_dev(x), out)
    check(to_host(out), expect, TOL[prec], f"{name} {op} {prec}")


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16", "i16"])
@pytest.mark.parametrize("op", ["D", "NORMAL", "MHATDAG", "HOP"])
def test_op_tiny_sites(ctx, prec, op):
    """Sites whose magnitude spans 1 down to 1e-60 (far below the FP32
    range), as at the front of a point-source solve: the per-site scale must
    neither overflow nor turn the tiny sites into NaN."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, "c1")
    x = S.random_spinor(act.lattice, act.L5, 300 + OPS.index(op))
    rng = np.random.default_rng(17)
    expo = rng.integers(0, 61, size=x.shape[:5]).astype(np.float64)
    x = x * (10.0 ** -expo)[..., None, None]
    expect = _oracle(op, U, x, oact)
    out = empty_like_dev(x.shape)
    ctx.dslash(g, act, getattr(M, "OP_" + op), prec, to_dev(x), out)
    got = to_host(out)
    assert np.isfinite(got).all()
    # norm-wise only: the element-wise bar relative to the largest site is
    # meaningless when site magnitudes span 60 decades
    err = rel(got, expect)
    log(f"   tiny sites {op} {prec}: norm-wise {err:.2e} (bar {TOL[prec]:.0e})")
    assert err < TOL[prec], err


def test_multi_rhs_dslash_matches_single(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, "tiles")
    n = 3
    x = S.random_spinor(act.lattice, act.L5, 300, nrhs=n)
    out = empty_like_dev(x.shape)
    ctx.dslash(g, act, M.OP_NORMAL, "f64", to_dev(x), out, nrhs=n)
    got = to_host(out)
    for r in range(n):
        one = empty_like_dev(x.shape[1:])
        ctx.dslash(g, act, M.OP_NORMAL, "f64", to_dev(x[r]), one)
        assert np.array_equal(to_host(one), got[r])


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_traversal_orders_bitwise(ctx, prec, monkeypatch):
    """The workgroup traversal (linear, blocked in t, cut into y-bands) only
    reorders whole workgroups: every order gives bitwise the same field."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, "banded")
    x = S.random_spinor(act.lattice, act.L5, 400)
    outs = []
    for bt, yb in ((0, 1), (2, 1), (4, 1), (2, 8), (4, 4), (4, 2)):
        monkeypatch.setenv("MDWF_BT", str(bt))
        monkeypatch.setenv("MDWF_YB", str(yb))
        log(f"[op] traversal bt={bt} yb={yb} {prec}")
        out = empty_like_dev(x.shape)
        ctx.dslash(g, act, M.OP_NORMAL, prec, to_dev(x), out)
        outs.append(to_host(out))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    check(outs[0], _oracle("NORMAL", U, x, oact), TOL[prec], f"traversal NORMAL {prec}")


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "i16"])
def test_streaming_stores_bitwise(ctx, prec, monkeypatch):
    """Streaming (non-temporal) stores change where the written lines live in
    the caches, never their values."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, "banded")
    x = S.random_spinor(act.lattice, act.L5, 410)
    outs = []
    for nt in ("0", "1"):
        monkeypatch.setenv("MDWF_NT", nt)
        out = empty_like_dev(x.shape)
        ctx.dslash(g, act, M.OP_NORMAL, prec, to_dev(x), out)
        outs.append(to_host(out))
    assert np.array_equal(outs[0], outs[1])


def test_gpu_identities(ctx):
    """Adjointness and gamma5-hermiticity measured on the GPU operators."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, "c1")
    x = S.random_spinor(act.lattice, act.L5, 400)
    y = S.random_spinor(act.lattice, act.L5, 401)

    def ap(op, v):
        out = empty_like_dev(v.shape)
        ctx.dslash(g, act, op, "f64", to_dev(v), out)
        return to_host(out)

    a = np.vdot(x, ap(M.OP_D, y))
    b = np.vdot(ap(M.OP_DDAG, x), y)
    assert abs(a - b) < 1e-12 * abs(a)
    Me = O.parity_mask(oact, 0)
    a = np.vdot(Me * x, ap(M.OP_MHAT, y))
    b = np.vdot(ap(M.OP_MHATDAG, x), Me * y)
    assert abs(a - b) < 1e-12 * abs(a)
    g5 = lambda v: np.einsum("ij,...jc->...ic", O.GAMMA5, v)
    assert rel(ap(M.OP_HOPDAG, x), g5(ap(M.OP_HOP, g5(x)))) < 1e-14


def test_gauge_covariance_gpu(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, "tiles")
    gt = S.random_gauge_transform(act.lattice, 9)
    Ug = O.gauge_transform_links(U, gt)
    gg = ctx.gauge_load(act.lattice, Ug)
    x = S.random_spinor(act.lattice, act.L5, 500)
    out1 = empty_like_dev(x.shape)
    out2 = empty_like_dev(x.shape)
    ctx.dslash(gg, act, M.OP_D, "f64", to_dev(O.gauge_transform_spinor(x, gt)), out1)
    ctx.dslash(g, act, M.OP_D, "f64", to_dev(x), out2)
    assert rel(to_host(out1), O.gauge_transform_spinor(to_host(out2), gt)) < 1e-13
    gg.free()


def test_sources_bitwise(ctx):
    from paper_1810_01609_amd import mdwf as M

    for name in ("c1", "ragged"):
        U, act, oact, g = _setup(ctx, name)
        eta = empty_like_dev(act.spinor_shape())
        ctx.source_z2(act, 1002, 3, eta)
        assert np.array_equal(to_host(eta), O.z2_source(oact, 1002, rhs=3))
        for spin in range(4):
            ctx.source_point(act, (1, 0, 1, 1), spin, 2, eta)
            assert np.array_equal(to_host(eta), O.point_source(oact, (1, 0, 1, 1), spin, 2))


def test_dslash_rejects_bad_arguments(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact, g = _setup(ctx, "c1")
    x = empty_like_dev(act.spinor_shape())
    bad = M.Action.make((4, 4, 4, 4), 8)  # lattice differs from the gauge field
    with pytest.raises(M.MDWFError) as e:
        ctx.dslash(g, bad, M.OP_D, "f64", empty_like_dev(bad.spinor_shape()), empty_like_dev(bad.spinor_shape()))
    assert e.value.status == M.EINVAL
    assert "lattice" in str(e.value)
    with pytest.raises(M.MDWFError):
        ctx.dslash(g, act, M.OP_D, "f64", x, x)  # in == out
    with pytest.raises(M.MDWFError):
        ctx.dslash(g, act, 99, "f64", x, empty_like_dev(act.spinor_shape()))
