"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test states which part of the oracle it pins.  Lattices are tiny so the
whole module runs in well under a minute on one core.
"""
import os

import numpy as np
import pytest

import mdwf_synth as S
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _act(L=(2, 2, 2, 4), L5=4, **kw):
    p = dict(b5=1.5, c5=0.5, M5=1.3, mq=0.05)
    p.update(kw)
    return O.Action(L, L5, **p)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# --------------------------------------------------------------------------
# Gamma basis (pins the chiral reading and the projectors)
# --------------------------------------------------------------------------
def test_gamma_algebra():
    for m in range(4):
        assert np.allclose(O.GAMMA[m], O.GAMMA[m].conj().T)
        for n in range(4):
            ac = O.GAMMA[m] @ O.GAMMA[n] + O.GAMMA[n] @ O.GAMMA[m]
            assert np.allclose(ac, 2.0 * (m == n) * np.eye(4))
    assert np.allclose(O.GAMMA5, np.diag([1, 1, -1, -1]))
    assert np.allclose(O.PPLUS @ O.PPLUS, O.PPLUS)
    assert np.allclose(O.PPLUS + O.PMINUS, np.eye(4))


# --------------------------------------------------------------------------
# P1: free field, momentum space.  Textbook Wilson kernel
#   D_W(p) = sum_mu (1 - cos p_mu) - M5 + i sum_mu gamma_mu sin p_mu
# and the Moebius 5D structure; pins H (signs, gammas), BCs and P5.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("antiperiodic", [True, False])
def test_free_field_plane_wave(antiperiodic):
    act = _act(L=(4, 2, 2, 4), L5=3, t_antiperiodic=antiperiodic)
    Lx, Ly, Lz, Lt = act.L
    U = S.unit_gauge(act.L)
    rng = np.random.default_rng(3)
    n = (1, 1, 0, 2)
    tw = 0.5 if antiperiodic else 0.0
    p = (2 * np.pi * n[0] / Lx, 2 * np.pi * n[1] / Ly, 2 * np.pi * n[2] / Lz, 2 * np.pi * (n[3] + tw) / Lt)
    chi = rng.standard_normal((act.L5, 4, 3)) + 1j * rng.standard_normal((act.L5, 4, 3))
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = phase[None, :, :, :, :, None, None] * chi[:, None, None, None, None, :, :]
    out = O.dirac(U, psi, act)
    # closed form, written independently of the oracle's projector form
    DW = (sum(1 - np.cos(pm) for pm in p) - act.M5) * np.eye(4) + 1j * sum(
        O.GAMMA[m] * np.sin(p[m]) for m in range(4))
    L5 = act.L5
    Pp, Pm = np.diag([1, 1, 0, 0]), np.diag([0, 0, 1, 1])
    P5 = np.zeros((4 * L5, 4 * L5), dtype=complex)
    for s in range(L5):
        # P- psi_{s+1} with P- psi_{L5} = -mq P- psi_0 ; P+ psi_{s-1} with P+ psi_{-1} = -mq P+ psi_{L5-1}
        sp, cp = ((s + 1), 1.0) if s + 1 < L5 else (0, -act.mq)
        sm, cm = ((s - 1), 1.0) if s >= 1 else (L5 - 1, -act.mq)
        P5[4 * s:4 * s + 4, 4 * sp:4 * sp + 4] += cp * Pm
        P5[4 * s:4 * s + 4, 4 * sm:4 * sm + 4] += cm * Pp
    DWb = np.kron(np.eye(L5), DW)
    I = np.eye(4 * L5)
    Dp = act.b5 * DWb + I + (act.c5 * DWb - I) @ P5
    expect = np.einsum("ab,bc->ac", Dp, chi.reshape(4 * L5, 3)).reshape(L5, 4, 3)
    expect = phase[None, :, :, :, :, None, None] * expect[:, None, None, None, None, :, :]
    assert _rel(out, expect) < 1e-13


# --------------------------------------------------------------------------
# P2: free-field solution (FFT + per-momentum 4L5 x 4L5 solves) equals the
# even-odd CGNR solution; pins prep, M^, M^dag, CG and reconstruction.
# --------------------------------------------------------------------------
def test_free_field_solution_matches_eo_cg():
    act = _act(L=(4, 4, 2, 4), L5=4, mq=0.1)
    U = S.unit_gauge(act.L)
    eta = O.point_source(act, (1, 2, 0, 3), spin=2, colour=1)
    psi_ff = O.free_field_solve(eta, act)
    psi_cg, info = O.solve(U, eta, act, tol=1e-12, max_iter=3000)
    assert _rel(psi_cg, psi_ff) < 1e-9
    assert _rel(O.dirac(U, psi_ff, act), eta) < 1e-12


# --------------------------------------------------------------------------
# P3: gamma5-hermiticity of the Wilson hop and kernel.
# --------------------------------------------------------------------------
def test_gamma5_hermiticity():
    act = _act()
    U = S.gauge_field(act.L, 0.3, 1)
    psi = S.random_spinor(act.L, act.L5, 11)
    chi = S.random_spinor(act.L, act.L5, 12)
    g5 = lambda v: np.einsum("ij,...jc->...ic", O.GAMMA5, v)
    # H^dag = gamma5 H gamma5 as an inner-product identity
    lhs = O.vdot(chi, O.hop(U, psi, act))
    rhs = O.vdot(g5(O.hop(U, g5(chi), act)), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the sign-flipped hop is gamma5 H gamma5
    assert _rel(O.hop_dag(U, psi, act), g5(O.hop(U, g5(psi), act))) < 1e-14


# --------------------------------------------------------------------------
# P4 / P5: Gamma5 = gamma5 R5 symmetry (Shamir: of D; Moebius: of D M_phi^-1).
# --------------------------------------------------------------------------
def _Gamma5(v):
    return np.einsum("ij,...jc->...ic", O.GAMMA5, v[::-1])


@pytest.mark.parametrize("c5,target", [(0.0, "D"), (0.5, "DMphiInv")])
def test_Gamma5_symmetry(c5, target):
    act = _act(b5=1.0 if c5 == 0.0 else 1.5, c5=c5)
    U = S.gauge_field(act.L, 0.3, 2)
    psi = S.random_spinor(act.L, act.L5, 13)
    chi = S.random_spinor(act.L, act.L5, 14)
    if target == "D":
        op = lambda v: O.dirac(U, v, act)
    else:
        L5 = act.L5
        Sup, Sdn = O.fifth_matrices(L5, act.mq)
        Ap_inv = np.linalg.inv(act.b5 * np.eye(L5) + act.c5 * Sdn)
        Am_inv = np.linalg.inv(act.b5 * np.eye(L5) + act.c5 * Sup)
        Pp, Pm = O.PPLUS, O.PMINUS

        def mphi_inv(v):
            up = np.einsum("st,t...->s...", Ap_inv, np.einsum("ij,...jc->...ic", Pp, v))
            dn = np.einsum("st,t...->s...", Am_inv, np.einsum("ij,...jc->...ic", Pm, v))
            return up + dn
        op = lambda v: O.dirac(U, mphi_inv(v), act)
    # op^dag = Gamma5 op Gamma5  <=>  <chi, op psi> = <Gamma5 op Gamma5 chi, psi>
    lhs = O.vdot(chi, op(psi))
    rhs = O.vdot(_Gamma5(op(_Gamma5(chi))), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_moebius_D_is_not_Gamma5_hermitian():
    """With c5 != 0, D itself breaks the symmetry (so the M_phi placement matters)."""
    act = _act()
    U = S.gauge_field(act.L, 0.3, 2)
    psi = S.random_spinor(act.L, act.L5, 13)
    chi = S.random_spinor(act.L, act.L5, 14)
    lhs = O.vdot(chi, O.dirac(U, psi, act))
    rhs = O.vdot(_Gamma5(O.dirac(U, _Gamma5(chi), act)), psi)
    assert abs(lhs - rhs) > 1e-3 * abs(lhs)


# --------------------------------------------------------------------------
# P6: adjointness against the dense conjugate transpose.
# --------------------------------------------------------------------------
def test_dagger_is_dense_conjugate_transpose():
    act = _act(L=(2, 2, 2, 2), L5=3)
    U = S.gauge_field(act.L, 0.3, 3)
    D = O.dense_matrix(lambda v: O.dirac(U, v, act), act.shape5)
    Dd = O.dense_matrix(lambda v: O.dirac_dag(U, v, act), act.shape5)
    assert np.abs(Dd - D.conj().T).max() < 1e-13
    Me = O.parity_mask(act, 0)
    M = O.dense_matrix(lambda v: O.mhat(U, Me * v, act), act.shape5)
    Md = O.dense_matrix(lambda v: O.mhat_dag(U, Me * v, act), act.shape5)
    assert np.abs(Md - M.conj().T).max() < 1e-13


def test_adjointness_random_vectors():
    act = _act(L=(4, 2, 2, 4), L5=5)
    U = S.gauge_field(act.L, 0.3, 4)
    x = S.random_spinor(act.L, act.L5, 15)
    y = S.random_spinor(act.L, act.L5, 16)
    a = O.vdot(x, O.dirac(U, y, act))
    b = O.vdot(O.dirac_dag(U, x, act), y)
    assert abs(a - b) < 1e-12 * abs(a)
    Me = O.parity_mask(act, 0)
    a = O.vdot(Me * x, O.mhat(U, Me * y, act))
    b = O.vdot(O.mhat_dag(U, Me * x, act), Me * y)
    assert abs(a - b) < 1e-12 * abs(a)


# --------------------------------------------------------------------------
# P7: gauge covariance of D and of the solution.
# --------------------------------------------------------------------------
def test_gauge_covariance():
    act = _act(L=(4, 2, 2, 4), L5=4)
    U = S.gauge_field(act.L, 0.3, 5)
    g = S.random_gauge_transform(act.L, 6)
    Ug = O.gauge_transform_links(U, g)
    psi = S.random_spinor(act.L, act.L5, 17)
    lhs = O.dirac(Ug, O.gauge_transform_spinor(psi, g), act)
    rhs = O.gauge_transform_spinor(O.dirac(U, psi, act), g)
    assert _rel(lhs, rhs) < 1e-13
    eta = O.z2_source(act, 9)
    sol, _ = O.solve(U, eta, act, tol=1e-12, max_iter=3000)
    solg, _ = O.solve(Ug, O.gauge_transform_spinor(eta, g), act, tol=1e-12, max_iter=3000)
    assert _rel(solg, O.gauge_transform_spinor(sol, g)) < 1e-9


# --------------------------------------------------------------------------
# P8: L5 = 1 reduces to a 4D Wilson operator (b5 - c5 mq) D_W + (1 + mq).
# --------------------------------------------------------------------------
def test_L5_one_reduces_to_wilson():
    act = _act(L5=1, mq=0.07)
    U = S.gauge_field(act.L, 0.3, 7)
    psi = S.random_spinor(act.L, 1, 18)
    expect = (act.b5 - act.c5 * act.mq) * O.dirac_wilson(U, psi, act) + (1 + act.mq) * psi
    assert _rel(O.dirac(U, psi, act), expect) < 1e-14


# --------------------------------------------------------------------------
# P9: M5^-1.  Closed form sum_k (-kappa)^k S^k / (alpha (1 + mq (-kappa)^L5))
# and the O(L5) recurrence both equal the oracle's dense inverse.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L5", [1, 2, 5, 8, 12, 16])
def test_m5_inverse_closed_form_and_recurrence(L5):
    act = _act(L5=L5, mq=0.05)
    alpha = act.b5 * (4 - act.M5) + 1
    beta = act.c5 * (4 - act.M5) - 1
    kappa = beta / alpha
    psi = S.random_spinor(act.L, L5, 19)
    ref = O.m5_inv(psi, act)
    assert _rel(O.m5(ref, act), psi) < 1e-14
    # closed form
    Sup, Sdn = O.fifth_matrices(L5, act.mq)
    c = alpha * (1 + act.mq * (-kappa) ** L5)
    Ap = sum((-kappa) ** k * np.linalg.matrix_power(Sdn, k) for k in range(L5)) / c
    Am = sum((-kappa) ** k * np.linalg.matrix_power(Sup, k) for k in range(L5)) / c
    up = np.einsum("st,t...->s...", Ap, np.einsum("ij,...jc->...ic", O.PPLUS, psi))
    dn = np.einsum("st,t...->s...", Am, np.einsum("ij,...jc->...ic", O.PMINUS, psi))
    assert _rel(up + dn, ref) < 1e-14
    # recurrence on the P+ half (forward in s) and P- half (backward in s)
    xp = np.einsum("ij,...jc->...ic", O.PPLUS, psi)
    xm = np.einsum("ij,...jc->...ic", O.PMINUS, psi)
    cc = 1 + act.mq * (-kappa) ** L5
    yp = np.zeros_like(xp)
    yp[0] = (xp[0] + sum((-kappa) ** k * (-act.mq) * xp[L5 - k] for k in range(1, L5))) / cc
    for s in range(1, L5):
        yp[s] = xp[s] - kappa * yp[s - 1]
    ym = np.zeros_like(xm)
    ym[L5 - 1] = (xm[L5 - 1] + sum((-kappa) ** k * (-act.mq) * xm[k - 1] for k in range(1, L5))) / cc
    for s in range(L5 - 2, -1, -1):
        ym[s] = xm[s] - kappa * ym[s + 1]
    assert _rel((yp + ym) / alpha, ref) < 1e-14


# --------------------------------------------------------------------------
# P10: D = M5 - 1/2 H M_phi, [M5, M_phi] = 0, both are 4D-site-local.
# --------------------------------------------------------------------------
def test_decomposition():
    act = _act()
    U = S.gauge_field(act.L, 0.3, 8)
    psi = S.random_spinor(act.L, act.L5, 20)
    d = O.m5(psi, act) - 0.5 * O.hop(U, O.m_phi(psi, act), act)
    assert _rel(O.dirac(U, psi, act), d) < 1e-14
    assert _rel(O.m5(O.m_phi(psi, act), act), O.m_phi(O.m5(psi, act), act)) < 1e-15
    Me, Mo = O.parity_mask(act, 0), O.parity_mask(act, 1)
    assert np.abs(Mo * O.m5(Me * psi, act)).max() == 0.0
    assert np.abs(Mo * O.m_phi(Me * psi, act)).max() == 0.0


# --------------------------------------------------------------------------
# P11: brute force.  Even-odd CGNR + reconstruction equals a dense LU solve.
# --------------------------------------------------------------------------
def test_eo_solve_equals_dense_solve():
    act = _act(L=(2, 2, 2, 4), L5=4)
    U = S.gauge_field(act.L, 0.3, 1)
    eta = O.z2_source(act, 7)
    psi_cg, info = O.solve(U, eta, act, tol=1e-13, max_iter=3000)
    psi_d = O.dense_solve(U, eta, act)
    assert _rel(psi_cg, psi_d) < 1e-11
    assert info["rel_res_full"] < 1e-12


# --------------------------------------------------------------------------
# P12: CG invariants: the A-norm error decreases monotonically and the
# recursive residual tracks the true one.
# --------------------------------------------------------------------------
def test_cg_invariants():
    act = _act(L=(2, 2, 2, 4), L5=4)
    U = S.gauge_field(act.L, 0.3, 1)
    eta = O.z2_source(act, 7)
    eta_hat = O.prep_source(U, eta, act)
    Me = O.parity_mask(act, 0)
    A = O.dense_matrix(lambda v: O.normal_op(U, Me * v, act), act.shape5)
    b = O.mhat_dag(U, eta_hat, act)
    idx = np.flatnonzero(np.broadcast_to(Me, act.shape5).ravel())
    Ae = A[np.ix_(idx, idx)]
    xs = np.linalg.solve(Ae, b.ravel()[idx])
    hist = []
    x, it = O.cgnr(U, eta_hat, act, tol=1e-12, max_iter=3000, history=hist)
    errs = []
    for (_, rr, xk) in hist:
        e = xk.ravel()[idx] - xs
        errs.append(np.sqrt(np.real(np.vdot(e, Ae @ e))))
    errs = np.array(errs)
    assert np.all(np.diff(errs) <= 1e-12 * errs[0])
    assert np.abs(x.ravel()[idx] - xs).max() / np.abs(xs).max() < 1e-10
    # recursive vs recomputed residual at the last step
    r_true = np.sqrt(O.norm2(b - O.normal_op(U, x, act)) / O.norm2(b))
    assert r_true < 1e-12


# --------------------------------------------------------------------------
# P13: synthetic gauge data are SU(3).
# --------------------------------------------------------------------------
def test_gauge_is_su3():
    U = S.gauge_field((4, 4, 4, 8), 0.3, 1)
    I = np.eye(3)
    err = np.abs(np.conj(np.swapaxes(U, -1, -2)) @ U - I).max()
    assert err < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # rows 0 and 1 determine row 2 = conj(row0 x row1)
    r2 = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    assert np.abs(r2 - U[..., 2, :]).max() < 1e-14


# --------------------------------------------------------------------------
# Sources: SplitMix64 against its published test vector; Z2 noise values;
# wall injection puts a spin-0 (P+) source only on the last slice.
# --------------------------------------------------------------------------
def test_splitmix64_golden():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) if l.strip() and not l.startswith("#")]
    assert [O.splitmix64(1234567, k) for k in range(len(vals))] == vals


def test_z2_noise_vectorised_matches_scalar():
    act = _act(L=(2, 2, 2, 2), L5=2)
    xi = O.z2_noise(act, 1234567, rhs=1)
    flat = xi.ravel()
    n = flat.size
    for k in range(n):
        z = O.splitmix64(1234567, n + k)
        expect = ((-1.0 if z & 1 else 1.0) + 1j * (-1.0 if z & 2 else 1.0)) * 0.7071067811865476
        assert flat[k] == expect
    assert np.allclose(np.abs(flat), 1.0)
    assert 0.7071067811865476 == float.fromhex('0x1.6a09e667f3bcdp-1')  # nearest double to 1/sqrt(2)


def test_point_source_wall_injection():
    act = _act(L5=6)
    eta = O.point_source(act, (1, 0, 1, 2), spin=0, colour=2)
    nz = np.argwhere(eta != 0)
    assert nz.shape == (1, 7)
    assert tuple(nz[0]) == (act.L5 - 1, 2, 1, 0, 1, 0, 2)
    eta = O.point_source(act, (0, 0, 0, 0), spin=3, colour=0)
    assert tuple(np.argwhere(eta != 0)[0]) == (0, 0, 0, 0, 0, 3, 0)


def test_sampled_dirac_matches_full():
    act = _act(L=(4, 2, 2, 4), L5=5)
    U = S.gauge_field(act.L, 0.3, 9)
    psi = S.random_spinor(act.L, act.L5, 21)
    full = O.dirac(U, psi, act)
    sites = [(0, 0, 0, 0, 0), (4, 3, 1, 1, 3), (2, 0, 1, 0, 1), (4, 0, 0, 1, 0)]
    got = O.dirac_at_sites(U, psi, act, sites)
    for k, (s, t, z, y, x) in enumerate(sites):
        assert _rel(got[k], full[s, t, z, y, x]) < 1e-14


# --------------------------------------------------------------------------
# Feynman-Hellmann sequential propagator (P14-P16).
# --------------------------------------------------------------------------
def test_gamma_products_clifford():
    """The 16 products of gamma matrices: mask 15 is the chiral gamma5
    diag(1,1,-1,-1) written out, each squares to +-1, and they are
    orthogonal, Tr(G_a^dag G_b) = 4 delta_ab (a basis of 4x4 matrices)."""
    assert np.array_equal(O.gamma_product(15), np.diag([1, 1, -1, -1]).astype(np.complex128))
    assert np.array_equal(O.gamma_product(0), np.eye(4, dtype=np.complex128))
    Gs = [O.gamma_product(m) for m in range(16)]
    for m, G in enumerate(Gs):
        sq = G @ G
        assert np.allclose(sq, np.eye(4)) or np.allclose(sq, -np.eye(4)), m
        # a signed permutation with entries in {+-1, +-i}
        assert np.count_nonzero(G) == 4 and np.allclose(np.abs(G[G != 0]), 1.0)
    T = np.array([[np.trace(a.conj().T @ b) for b in Gs] for a in Gs])
    assert np.allclose(T, 4 * np.eye(16))
    # single gammas are the basis matrices themselves
    for mu in range(4):
        assert np.array_equal(O.gamma_product(1 << mu), O.GAMMA[mu])


def test_propagator_4d_inverts_wall_injection():
    """Reading the walls back, q = P- eta_0 + P+ eta_{L5-1}, returns the 4D
    field a source was made from (for L5 = 1 as well)."""
    for L5 in (1, 2, 5):
        act = _act(L=(2, 2, 2, 4), L5=L5)
        xi = S.random_spinor(act.L, 1, 3)[0]
        assert np.array_equal(O.propagator_4d(O.wall_inject(xi, act), act), xi)


@pytest.mark.parametrize("mask", [0, 11, 15])
def test_feynman_hellmann_derivative(mask):
    """The Feynman-Hellmann theorem on a 2^3x4, L5=4 lattice: with the current
    J = inject o Gamma o extract added to the action, D(l) = D + l J,
    d/dl D(l)^-1 eta = -D^-1 J D^-1 eta.  The central difference of dense
    solves at l = +-1e-5 equals minus the sequential propagator; the
    even-odd CG of fh_solve equals the dense sequential solve."""
    act = _act(L=(2, 2, 2, 4), L5=4)
    U = S.gauge_field(act.L, 0.3, 2)
    shape = act.shape5
    Dm = O.dense_matrix(lambda v: O.dirac(U, v, act), shape)
    Jm = O.dense_matrix(lambda v: O.fh_operator(v, act, mask), shape)
    eta = O.point_source(act, (0, 0, 0, 0), 1, 2).ravel()
    psi = np.linalg.solve(Dm, eta)
    psi_fh = np.linalg.solve(Dm, Jm @ psi)
    lam = 1e-5
    fd = (np.linalg.solve(Dm + lam * Jm, eta) - np.linalg.solve(Dm - lam * Jm, eta)) / (2 * lam)
    assert _rel(-fd, psi_fh) < 1e-7
    got, _ = O.fh_solve(U, psi.reshape(shape), act, mask, tol=1e-13)
    assert _rel(got.ravel(), psi_fh) < 1e-10


# --------------------------------------------------------------------------
# Physical 4D propagator of the Moebius action and the Feynman-Hellmann
# sequential propagator built from it (P17-P18).
# --------------------------------------------------------------------------
def _dense_4d_propagator(U, act, source):
    """Dense 4D map xi -> R D^-1 source(xi) through the 5D operator."""
    Lx, Ly, Lz, Lt = act.L
    shape4 = (Lt, Lz, Ly, Lx, 4, 3)
    n4 = int(np.prod(shape4))
    D5 = O.dense_matrix(lambda v: O.dirac(U, v, act), act.shape5)
    B = np.zeros((D5.shape[0], n4), dtype=np.complex128)
    e = np.zeros(n4, dtype=np.complex128)
    for k in range(n4):
        e[k] = 1.0
        B[:, k] = source(e.reshape(shape4)).ravel()
        e[k] = 0.0
    X = np.linalg.solve(D5, B)
    return np.stack([O.propagator_4d(X[:, k].reshape(act.shape5), act).ravel() for k in range(n4)], axis=1)


@pytest.mark.parametrize("b5,c5", [(1.0, 0.0), (1.5, 0.5)])
@pytest.mark.parametrize("L5", [1, 2, 4])
def test_physical_propagator_is_truncated_overlap(b5, c5, L5):
    """The 4D propagator read off the walls of D^-1 (1 - c5 D_W) inject(xi)
    equals (D_eff^-1 - 1) / (1 - mq) xi, D_eff the truncated overlap operator
    of the Moebius kernel H_M = g5 (b5 + c5) D_W / (2 + (b5 - c5) D_W),
    built from dense 4D matrix functions with no 5D operator involved
    (Shamir for c5 = 0, Moebius for c5 = 0.5; L5 = 1, 2, 4 on 2^3 x 4).
    Without the (1 - c5 D_W) factor the Moebius case fails."""
    act = O.Action((2, 2, 2, 4), L5, b5, c5, 1.3, 0.05)
    U = S.gauge_field(act.L, 0.3, 3)
    Sref = O.effective_propagator_4d(U, act)
    Sg = _dense_4d_propagator(U, act, lambda xi: O.physical_source(U, xi, act))
    assert _rel(Sg, Sref) < 1e-12, _rel(Sg, Sref)
    if c5 != 0.0 and L5 > 1:
        Sbare = _dense_4d_propagator(U, act, lambda xi: O.wall_inject_physical(xi, act))
        assert _rel(Sbare, Sref) > 0.1


def test_physical_source_shamir_limit_and_l5_one():
    """c5 = 0: the physical source is the plain opposite-wall injection; L5 = 1:
    both walls are slice 0 and the source is (1 - c5 D_W) xi."""
    U = S.gauge_field((2, 2, 2, 4), 0.3, 4)
    xi = S.random_spinor((2, 2, 2, 4), 1, 5)[0]
    sh = O.Action((2, 2, 2, 4), 5, 1.0, 0.0, 1.3, 0.05)
    assert np.array_equal(O.physical_source(U, xi, sh), O.wall_inject_physical(xi, sh))
    one = O.Action((2, 2, 2, 4), 1, 1.5, 0.5, 1.3, 0.05)
    want = xi - 0.5 * ((4.0 - 1.3) * xi - 0.5 * O.hop(U, xi[None], one)[0])
    assert _rel(O.physical_source(U, xi, one)[0], want) < 1e-15


@pytest.mark.parametrize("mask", [0, 11])
def test_physical_feynman_hellmann_is_s_gamma_s(mask):
    """The physical sequential propagator read off the second 5D solve equals
    S Gamma S xi with S the dense 4D truncated-overlap propagator: the current
    is inserted once, at every site, between two 4D propagators (the
    Feynman-Hellmann derivative of the 4D propagator with Gamma added to the
    4D action)."""
    act = O.Action((2, 2, 2, 4), 4, 1.5, 0.5, 1.3, 0.05)
    U = S.gauge_field(act.L, 0.3, 6)
    Sref = O.effective_propagator_4d(U, act)
    xi = S.random_spinor(act.L, 1, 8)[0]
    q, qfh = O.fh_solve_physical(U, xi, act, mask, tol=1e-13)
    G = np.kron(np.eye(xi.size // 12), np.kron(O.gamma_product(mask), np.eye(3)))
    assert _rel(q.ravel(), Sref @ xi.ravel()) < 1e-10
    assert _rel(qfh.ravel(), Sref @ (G @ (Sref @ xi.ravel()))) < 1e-10
