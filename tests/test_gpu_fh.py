"""Feynman-Hellmann sequential propagator on the GPU against the oracle:
the wall read-out and the current source are exact FP64 selections and
signed permutations (bit-exact), the sequential solve matches the oracle's
to the 1e-8 solution bar."""
import numpy as np
import pytest

import mdwf_synth as S
import oracle as O
from gpu_util import check, empty_like_dev, log, make_case, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1810_01609_amd import mdwf as M

    c = M.Context(0)
    yield c
    c.close()


SHAPES = [((4, 4, 4, 8), 8), ((6, 2, 2, 2), 3), ((4, 2, 2, 4), 1)]


@pytest.mark.parametrize("L,L5", SHAPES)
def test_propagator_4d_bitwise(ctx, L, L5):
    U, act, oact = make_case(L, L5, 0.05, 0.3, 1)
    nrhs = 2
    psi = S.random_spinor(L, L5, 41, nrhs=nrhs)
    q = empty_like_dev((nrhs,) + psi.shape[2:])
    ctx.propagator_4d(act, to_dev(psi), q, nrhs=nrhs)
    got = to_host(q)
    for r in range(nrhs):
        assert np.array_equal(got[r], O.propagator_4d(psi[r], oact))


@pytest.mark.parametrize("L,L5", SHAPES)
def test_current_source_bitwise(ctx, L, L5):
    U, act, oact = make_case(L, L5, 0.05, 0.3, 1)
    nrhs = 2
    q = S.random_spinor(L, 1, 43, nrhs=nrhs)[:, 0]
    for mask in range(16):
        eta = empty_like_dev((nrhs, L5) + q.shape[1:])
        eta.fill_(7.0)  # every entry must be written
        ctx.current_source(act, mask, to_dev(q), eta, nrhs=nrhs)
        got = to_host(eta)
        for r in range(nrhs):
            assert np.array_equal(got[r], O.current_source(q[r], oact, mask)), (mask, r)


@pytest.mark.parametrize("inner,mask", [("f32", 11), ("f16", 15), ("f64", 0)])
def test_sequential_solve_matches_oracle(ctx, inner, mask):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact = make_case((4, 4, 4, 8), 8, 0.05, 0.3, 1)
    g = ctx.gauge_load(act.lattice, U, precs=("f64", inner))
    eta = O.point_source(oact, (0, 0, 0, 0), 0, 0)
    psi_o, _ = O.solve(U, eta, oact, tol=1e-12)
    fh_o, _ = O.fh_solve(U, psi_o, oact, mask, tol=1e-12)
    opts = M.CGOpts.make(tol=1e-10, inner=inner)
    psi = empty_like_dev(eta.shape)
    ctx.solve(g, act, opts, to_dev(eta), psi)
    q = empty_like_dev(eta.shape[1:])
    ctx.propagator_4d(act, psi, q)
    eta2 = empty_like_dev(eta.shape)
    ctx.current_source(act, mask, q, eta2)
    fh = empty_like_dev(eta.shape)
    st = ctx.solve(g, act, opts, eta2, fh)[0]
    err = rel(to_host(fh), fh_o)
    log(f"[fh] {inner} mask {mask}: {st['iters']} it, err {err:.2e}")
    assert st["converged"] == 1
    assert err < 1e-8, err
    g.free()


def test_fh_rejects_bad_arguments(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact = make_case((4, 4, 4, 8), 8, 0.05, 0.3, 1)
    q = empty_like_dev((8, 4, 4, 4, 4, 3))
    eta = empty_like_dev(act.spinor_shape())
    with pytest.raises(M.MDWFError) as e:
        ctx.current_source(act, 16, q, eta)
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MDWFError):
        ctx.current_source(act, -1, q, eta)


@pytest.mark.parametrize("L,L5", SHAPES)
@pytest.mark.parametrize("c5", [0.5, 0.0])
def test_source_physical_matches_oracle(ctx, L, L5, c5):
    """The physical 4D-propagator source (1 - c5 D_W) inject(Gamma xi) against
    the oracle's, every current mask in one pass over two right-hand sides;
    FP64 on both sides (the library sums the hop's terms in its own order)."""
    from paper_1810_01609_amd import mdwf as M

    U = S.gauge_field(L, 0.3, 2)
    act = M.Action.make(L, L5, 1.5, c5, 1.3, 0.05)
    oact = O.Action(L, L5, 1.5, c5, 1.3, 0.05)
    g = ctx.gauge_load(L, U, precs=("f64",))
    nrhs = 2
    xi = S.random_spinor(L, 1, 47, nrhs=nrhs)[:, 0]
    for mask in (0, 1, 6, 11, 15):
        eta = empty_like_dev((nrhs, L5) + xi.shape[1:])
        eta.fill_(7.0)  # every entry must be written
        ctx.source_physical(g, act, to_dev(xi), eta, gamma_mask=mask, nrhs=nrhs)
        got = to_host(eta)
        for r in range(nrhs):
            check(got[r], O.physical_source(U, xi[r], oact, mask), 1e-14, f"physical source L5={L5} c5={c5} mask {mask}")
    g.free()


@pytest.mark.parametrize("inner,mask", [("f32", 11), ("f16", 15)])
def test_physical_fh_pair_matches_oracle(ctx, inner, mask):
    """The physical propagator q = S xi and the sequential one S Gamma S xi,
    each a GPU solve read off the walls, against the oracle's (solved to
    1e-12) at the 1e-8 solution bar."""
    from paper_1810_01609_amd import mdwf as M

    U, act, oact = make_case((4, 4, 4, 8), 8, 0.05, 0.3, 1)
    g = ctx.gauge_load(act.lattice, U, precs=("f64", inner))
    xi = np.zeros((8, 4, 4, 4, 4, 3), dtype=np.complex128)
    xi[0, 0, 0, 0, 0, 0] = 1.0  # point source, spin 0, colour 0, at the origin
    q_o, fh_o = O.fh_solve_physical(U, xi, oact, mask, tol=1e-12)
    opts = M.CGOpts.make(tol=1e-10, inner=inner)
    eta = empty_like_dev(act.spinor_shape())
    ctx.source_physical(g, act, to_dev(xi), eta)
    psi = empty_like_dev(act.spinor_shape())
    s1 = ctx.solve(g, act, opts, eta, psi)[0]
    q = empty_like_dev(xi.shape)
    ctx.propagator_4d(act, psi, q)
    eta2 = empty_like_dev(act.spinor_shape())
    ctx.source_physical(g, act, q, eta2, gamma_mask=mask)
    psi2 = empty_like_dev(act.spinor_shape())
    s2 = ctx.solve(g, act, opts, eta2, psi2)[0]
    qfh = empty_like_dev(xi.shape)
    ctx.propagator_4d(act, psi2, qfh)
    e1, e2 = rel(to_host(q), q_o), rel(to_host(qfh), fh_o)
    log(f"[fh-phys] {inner} mask {mask}: {s1['iters']}+{s2['iters']} it, q err {e1:.2e}, q_FH err {e2:.2e}")
    assert s1["converged"] == 1 and s2["converged"] == 1
    assert e1 < 1e-8 and e2 < 1e-8, (e1, e2)
    g.free()


def test_source_physical_rejects(ctx):
    from paper_1810_01609_amd import mdwf as M

    U, act, oact = make_case((4, 4, 4, 8), 8, 0.05, 0.3, 1)
    xi = empty_like_dev((8, 4, 4, 4, 4, 3))
    eta = empty_like_dev(act.spinor_shape())
    g = ctx.gauge_load(act.lattice, U, precs=("f64",))
    for mask in (-1, 16):
        with pytest.raises(M.MDWFError, match="gamma_mask"):
            ctx.source_physical(g, act, xi, eta, gamma_mask=mask)
    other = M.Action.make((4, 4, 4, 4), 8)
    with pytest.raises(M.MDWFError, match="differs"):
        ctx.source_physical(g, other, empty_like_dev((4, 4, 4, 4, 4, 3)), empty_like_dev(other.spinor_shape()))
    g.free()
