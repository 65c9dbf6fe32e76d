"""Plain FP64 NumPy oracle for the Moebius domain-wall fermion (MDWF) solve.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  The HIP path never imports it.

What it computes (paper, "Current State of the Art", Background and
Performance-related paragraphs): the propagator psi = D^{-1} eta of the
Moebius domain-wall Dirac operator D on an L^3 x T x L5 lattice with 3 colours
and 4 spins, obtained by conjugate gradient on the normal equations of the
red-black (even-odd) preconditioned operator.  The paper names this operator,
the preconditioning and the solver but writes none of them down, so the
definitions below follow the standard Moebius form (Brower, Neff, Orginos,
arXiv:1206.5214) with these readings:

* gamma matrices in the DeGrand-Rossi chiral basis, gamma5 = diag(1,1,-1,-1);
* periodic boundaries in x, y, z and antiperiodic in t;
* 5th-dimension walls carry -m_q: P- psi_{L5} := -m_q P- psi_0 and
  P+ psi_{-1} := -m_q P+ psi_{L5-1};
* even-odd by 4D parity, left Schur complement on the even sites;
* a 4D source xi enters the 5D source on the walls:
  eta_0 = P- xi, eta_{L5-1} = P+ xi.

Fields are complex128 arrays in the user layout ``[s][t][z][y][x][spin][col]``
(one right-hand side); gauge links are ``[t][z][y][x][mu][row][col]``.
Every function is written from its definition, loops over directions and
slices are explicit, and nothing is fused or reordered for speed.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "GAMMA", "GAMMA5", "PPLUS", "PMINUS", "IDENT4",
    "Action", "parity_mask", "hop", "hop_dag", "dirac_wilson",
    "p5", "p5_dag", "m_phi", "m_phi_dag", "m5", "m5_dag", "m5_inv", "m5_inv_dag",
    "fifth_matrices", "dirac", "dirac_dag",
    "hop_eo", "hop_oe", "mhat", "mhat_dag", "normal_op", "prep_source", "reconstruct",
    "cgnr", "solve", "dense_matrix", "dense_solve",
    "free_field_momentum_matrix", "free_field_solve",
    "point_source", "splitmix64", "z2_noise", "z2_source", "wall_inject",
    "gauge_transform_links", "gauge_transform_spinor",
    "dirac_at_sites", "vdot", "norm2",
    "gamma_product", "propagator_4d", "current_source", "fh_solve", "fh_operator",
    "wall_inject_physical", "dminus", "physical_source", "current_source_physical", "fh_solve_physical",
    "effective_propagator_4d",
]

# ---------------------------------------------------------------------------
# Gamma matrices: DeGrand-Rossi chiral basis (a reading; the paper is silent).
# mu = 0,1,2,3 <-> x,y,z,t.
# ---------------------------------------------------------------------------
_i = 1j
GAMMA = np.array(
    [
        [[0, 0, 0, _i], [0, 0, _i, 0], [0, -_i, 0, 0], [-_i, 0, 0, 0]],  # gamma_x
        [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],      # gamma_y
        [[0, 0, _i, 0], [0, 0, 0, -_i], [-_i, 0, 0, 0], [0, _i, 0, 0]],  # gamma_z
        [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],        # gamma_t
    ],
    dtype=np.complex128,
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
IDENT4 = np.eye(4, dtype=np.complex128)
PPLUS = 0.5 * (IDENT4 + GAMMA5)
PMINUS = 0.5 * (IDENT4 - GAMMA5)

# axis of direction mu in a spinor array [s][t][z][y][x][spin][col]
_SPIN_AXIS = {0: 4, 1: 3, 2: 2, 3: 1}
# axis of direction mu in a link array [t][z][y][x][mu][row][col] (after mu is taken)
_LINK_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


class Action:
    """Moebius domain-wall parameters for one solve.

    D = (b5 D_W + 1) + (c5 D_W - 1) P5, with D_W = (4 - M5) - H/2.
    """

    def __init__(self, L, L5, b5=1.5, c5=0.5, M5=1.3, mq=0.05, t_antiperiodic=True):
        self.L = tuple(int(v) for v in L)
        self.L5 = int(L5)
        self.b5 = float(b5)
        self.c5 = float(c5)
        self.M5 = float(M5)
        self.mq = float(mq)
        self.t_antiperiodic = bool(t_antiperiodic)

    @property
    def shape5(self):
        Lx, Ly, Lz, Lt = self.L
        return (self.L5, Lt, Lz, Ly, Lx, 4, 3)


def vdot(a, b):
    """<a, b> = sum conj(a) b over every index."""
    return np.vdot(a.ravel(), b.ravel())


def norm2(a):
    return float(np.real(vdot(a, a)))


def _spin(M, psi):
    """Apply a 4x4 spin matrix to a field [..][spin][col]."""
    return np.einsum("ij,...jc->...ic", M, psi)


# ---------------------------------------------------------------------------
# 4D hopping term (same on every 5th-dimension slice).
# (H psi)_s(x) = sum_mu (1 - g_mu) U_mu(x) psi_s(x+mu)
#                     + (1 + g_mu) U_mu(x-mu)^dag psi_s(x-mu)
# ---------------------------------------------------------------------------
def _shift(psi, mu, direction, act):
    """psi(x + direction*mu) on every site, with the time boundary sign.

    direction = +1 fetches the forward neighbour, -1 the backward one.  A hop
    that crosses the t boundary picks up -1 when the field is antiperiodic.
    """
    ax = _SPIN_AXIS[mu]
    out = np.roll(psi, -direction, axis=ax)
    if mu == 3 and act.t_antiperiodic:
        Lt = psi.shape[ax]
        sl = [slice(None)] * psi.ndim
        sl[ax] = Lt - 1 if direction == +1 else 0
        out[tuple(sl)] *= -1.0
    return out


def hop(U, psi, act: Action, sign: float = 1.0):
    """H psi with projectors (1 - sign*g_mu) forward, (1 + sign*g_mu) backward.

    sign = +1 is H; sign = -1 gives gamma5 H gamma5 = H^dag.
    """
    out = np.zeros_like(psi)
    for mu in range(4):
        Umu = U[..., mu, :, :]                                   # [t][z][y][x][a][b]
        # forward: U_mu(x) psi(x+mu)
        fwd = np.einsum("tzyxab,stzyxjb->stzyxja", Umu, _shift(psi, mu, +1, act))
        out += fwd - sign * _spin(GAMMA[mu], fwd)
        # backward: U_mu(x-mu)^dag psi(x-mu)
        Ub = np.roll(Umu, 1, axis=_LINK_AXIS[mu])                # U_mu(x - mu)
        bwd = np.einsum("tzyxba,stzyxjb->stzyxja", np.conj(Ub), _shift(psi, mu, -1, act))
        out += bwd + sign * _spin(GAMMA[mu], bwd)
    return out


def hop_dag(U, psi, act):
    return hop(U, psi, act, sign=-1.0)


def dirac_wilson(U, psi, act):
    """D_W psi = (4 - M5) psi - H psi / 2 (Wilson kernel with mass -M5)."""
    return (4.0 - act.M5) * psi - 0.5 * hop(U, psi, act)


# ---------------------------------------------------------------------------
# 5th dimension.  As L5 x L5 real matrices per chirality:
#   S_up: (S_up x)_s = x_{s+1}, (S_up x)_{L5-1} = -mq x_0
#   S_dn: (S_dn x)_s = x_{s-1}, (S_dn x)_0     = -mq x_{L5-1}
#   P5 = P- S_up + P+ S_dn ;  P5^dag = P- S_dn + P+ S_up  (S_up^T = S_dn)
#   M_phi = b5 + c5 P5 ;  M5 = alpha + beta P5 with alpha = b5(4-M5)+1,
#   beta = c5(4-M5)-1.
# ---------------------------------------------------------------------------
def fifth_matrices(L5, mq):
    """The two L5 x L5 wall-shift matrices (S_up, S_dn)."""
    S_up = np.zeros((L5, L5))
    S_dn = np.zeros((L5, L5))
    for s in range(L5):
        if s + 1 < L5:
            S_up[s, s + 1] = 1.0
        else:
            S_up[s, 0] = -mq
        if s - 1 >= 0:
            S_dn[s, s - 1] = 1.0
        else:
            S_dn[s, L5 - 1] = -mq
    return S_up, S_dn


def _apply_chiral(psi, A_plus, A_minus):
    """Apply L5 x L5 matrix A_plus on the P+ part and A_minus on the P- part."""
    up = np.einsum("st,t...->s...", A_plus, _spin(PPLUS, psi))
    dn = np.einsum("st,t...->s...", A_minus, _spin(PMINUS, psi))
    return up + dn


def _coeffs(act):
    alpha = act.b5 * (4.0 - act.M5) + 1.0
    beta = act.c5 * (4.0 - act.M5) - 1.0
    return alpha, beta


def _fifth_op(act, a, b, dag=False, inverse=False):
    """L5 x L5 matrices (for P+, for P-) of a*1 + b*P5 (or its transpose / inverse)."""
    S_up, S_dn = fifth_matrices(act.L5, act.mq)
    I = np.eye(act.L5)
    Ap = a * I + b * (S_up if dag else S_dn)
    Am = a * I + b * (S_dn if dag else S_up)
    if inverse:
        Ap, Am = np.linalg.inv(Ap), np.linalg.inv(Am)
    return Ap, Am


def p5(psi, act):
    return _apply_chiral(psi, *_fifth_op(act, 0.0, 1.0))


def p5_dag(psi, act):
    return _apply_chiral(psi, *_fifth_op(act, 0.0, 1.0, dag=True))


def m_phi(psi, act):
    return _apply_chiral(psi, *_fifth_op(act, act.b5, act.c5))


def m_phi_dag(psi, act):
    return _apply_chiral(psi, *_fifth_op(act, act.b5, act.c5, dag=True))


def m5(psi, act):
    return _apply_chiral(psi, *_fifth_op(act, *_coeffs(act)))


def m5_dag(psi, act):
    return _apply_chiral(psi, *_fifth_op(act, *_coeffs(act), dag=True))


def m5_inv(psi, act):
    """M5^{-1}: the inverse of the dense L5 x L5 chiral blocks (library inverse)."""
    return _apply_chiral(psi, *_fifth_op(act, *_coeffs(act), inverse=True))


def m5_inv_dag(psi, act):
    return _apply_chiral(psi, *_fifth_op(act, *_coeffs(act), dag=True, inverse=True))


# ---------------------------------------------------------------------------
# Full 5D operator (Brower-Neff-Orginos Moebius form).
# ---------------------------------------------------------------------------
def dirac(U, psi, act):
    """D psi = (b5 D_W + 1) psi + (c5 D_W - 1) P5 psi."""
    p = p5(psi, act)
    return act.b5 * dirac_wilson(U, psi, act) + psi + act.c5 * dirac_wilson(U, p, act) - p


def dirac_dag(U, psi, act):
    """D^dag psi = (b5 D_W^dag + 1) psi + P5^dag (c5 D_W^dag - 1) psi.

    D_W^dag = (4 - M5) - H^dag / 2 with H^dag = gamma5 H gamma5.
    """
    dw_dag = (4.0 - act.M5) * psi - 0.5 * hop_dag(U, psi, act)
    return act.b5 * dw_dag + psi + p5_dag(act.c5 * dw_dag - psi, act)


# ---------------------------------------------------------------------------
# Even-odd (red-black) preconditioning by 4D parity.
# D = [[M5, -H_eo M_phi / 2], [-H_oe M_phi / 2, M5]].
# Half-fields are kept as full arrays with the other parity zero.
# ---------------------------------------------------------------------------
def parity_mask(act, parity):
    Lx, Ly, Lz, Lt = act.L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    m = ((x + y + z + t) % 2 == parity).astype(np.float64)
    return m[None, :, :, :, :, None, None]


def hop_eo(U, psi, act, sign=1.0):
    """H_eo: odd sites of psi -> even sites."""
    return parity_mask(act, 0) * hop(U, parity_mask(act, 1) * psi, act, sign)


def hop_oe(U, psi, act, sign=1.0):
    """H_oe: even sites of psi -> odd sites."""
    return parity_mask(act, 1) * hop(U, parity_mask(act, 0) * psi, act, sign)


def mhat(U, x, act):
    """M^ x = x - 1/4 M5^-1 H_eo M_phi M5^-1 H_oe M_phi x   (x on even sites)."""
    t = m_phi(x, act)
    t = hop_oe(U, t, act)
    t = m5_inv(t, act)
    t = m_phi(t, act)
    t = hop_eo(U, t, act)
    t = m5_inv(t, act)
    return parity_mask(act, 0) * x - 0.25 * t


def mhat_dag(U, x, act):
    """M^dag x = x - 1/4 M_phi^T (g5 H_eo g5) M5^-T M_phi^T (g5 H_oe g5) M5^-T x."""
    t = m5_inv_dag(x, act)
    t = hop_oe(U, t, act, sign=-1.0)
    t = m_phi_dag(t, act)
    t = m5_inv_dag(t, act)
    t = hop_eo(U, t, act, sign=-1.0)
    t = m_phi_dag(t, act)
    return parity_mask(act, 0) * x - 0.25 * t


def normal_op(U, x, act):
    return mhat_dag(U, mhat(U, x, act), act)


def prep_source(U, eta, act):
    """eta^_e = M5^-1 (eta_e + 1/2 H_eo M_phi M5^-1 eta_o)."""
    eta_e = parity_mask(act, 0) * eta
    eta_o = parity_mask(act, 1) * eta
    t = hop_eo(U, m_phi(m5_inv(eta_o, act), act), act)
    return m5_inv(eta_e + 0.5 * t, act)


def reconstruct(U, psi_e, eta, act):
    """psi_o = M5^-1 (eta_o + 1/2 H_oe M_phi psi_e); returns the full psi."""
    eta_o = parity_mask(act, 1) * eta
    psi_o = m5_inv(eta_o + 0.5 * hop_oe(U, m_phi(psi_e, act), act), act)
    return parity_mask(act, 0) * psi_e + psi_o


# ---------------------------------------------------------------------------
# Conjugate gradient on the normal equations (plain FP64).
# ---------------------------------------------------------------------------
def cgnr(U, eta_hat, act, tol=1e-10, max_iter=100000, x0=None, history=None):
    """Solve M^dag M^ x = M^dag eta^ by CG.  Returns (x, iterations).

    Stops when sqrt(rho) <= tol*|b|, then recomputes r = b - A x and re-tests
    on that true residual, continuing if it is not yet met.
    """
    b = mhat_dag(U, eta_hat, act)
    bnorm = np.sqrt(norm2(b))
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - normal_op(U, x, act) if x0 is not None else b.copy()
    p = r.copy()
    rho = norm2(r)
    it = 0
    if bnorm == 0.0:
        return x, 0
    while it < max_iter:
        q = normal_op(U, p, act)
        pq = float(np.real(vdot(p, q)))
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rho_new = norm2(r)
        it += 1
        if history is not None:
            history.append((it, np.sqrt(rho_new) / bnorm, x.copy()))
        if np.sqrt(rho_new) <= tol * bnorm:
            r = b - normal_op(U, x, act)
            rho_new = norm2(r)
            if np.sqrt(rho_new) <= tol * bnorm:
                break
        beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
    return x, it


def solve(U, eta, act, tol=1e-10, max_iter=100000):
    """psi = D^-1 eta through even-odd CGNR; returns (psi, info dict)."""
    eta_hat = prep_source(U, eta, act)
    x, it = cgnr(U, eta_hat, act, tol=tol, max_iter=max_iter)
    psi = reconstruct(U, x, eta, act)
    res = eta - dirac(U, psi, act)
    info = dict(
        iters=it,
        rel_res_full=np.sqrt(norm2(res) / norm2(eta)),
        rel_res_normal=np.sqrt(
            norm2(mhat_dag(U, eta_hat, act) - normal_op(U, x, act)) / norm2(mhat_dag(U, eta_hat, act))
        ),
    )
    return psi, info


# ---------------------------------------------------------------------------
# Brute force on tiny lattices.
# ---------------------------------------------------------------------------
def dense_matrix(op, shape):
    """Dense matrix of a linear map on fields of the given shape (unit vectors)."""
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        e[k] = 1.0
        M[:, k] = op(e.reshape(shape)).ravel()
        e[k] = 0.0
    return M


def dense_solve(U, eta, act):
    """psi = D^-1 eta from a dense LU solve of the full 5D operator."""
    Dm = dense_matrix(lambda v: dirac(U, v, act), act.shape5)
    return np.linalg.solve(Dm, eta.ravel()).reshape(act.shape5)


# ---------------------------------------------------------------------------
# Free field (U = 1) in momentum space.
# A plane wave e^{ip.x} chi_s is an eigenvector of H with
#   H(p) = sum_mu [ (1 - g_mu) e^{ip_mu} + (1 + g_mu) e^{-ip_mu} ],
# p_i = 2 pi n_i / L_i, p_t = 2 pi (n_t + 1/2) / L_t when t is antiperiodic.
# ---------------------------------------------------------------------------
def _momenta(act):
    Lx, Ly, Lz, Lt = act.L
    tw = 0.5 if act.t_antiperiodic else 0.0
    return (2 * np.pi * np.arange(Lx) / Lx, 2 * np.pi * np.arange(Ly) / Ly,
            2 * np.pi * np.arange(Lz) / Lz, 2 * np.pi * (np.arange(Lt) + tw) / Lt)


def free_field_momentum_matrix(act, p):
    """(4 L5) x (4 L5) matrix of D at momentum p = (px, py, pz, pt) (colour-blind).

    Index order (s, spin).
    """
    Hp = np.zeros((4, 4), dtype=np.complex128)
    for mu in range(4):
        Hp += (IDENT4 - GAMMA[mu]) * np.exp(1j * p[mu]) + (IDENT4 + GAMMA[mu]) * np.exp(-1j * p[mu])
    DW = (4.0 - act.M5) * IDENT4 - 0.5 * Hp
    S_up, S_dn = fifth_matrices(act.L5, act.mq)
    P5 = np.kron(S_up, PMINUS) + np.kron(S_dn, PPLUS)
    I5 = np.eye(act.L5)
    DWb = np.kron(I5, DW)
    I = np.eye(4 * act.L5)
    return act.b5 * DWb + I + (act.c5 * DWb - I) @ P5


def free_field_solve(eta, act):
    """psi = D^-1 eta for U = 1: Fourier transform, 4L5 x 4L5 solve per momentum."""
    Lx, Ly, Lz, Lt = act.L
    L5 = act.L5
    tw = 0.5 if act.t_antiperiodic else 0.0
    t = np.arange(Lt)
    phase = np.exp(-1j * np.pi * 2 * tw * t / Lt)[None, :, None, None, None, None, None]
    # eta~(p) = sum_x e^{-ip.x} eta(x); the antiperiodic half-unit shift in p_t
    # becomes a phase on t before an ordinary FFT.
    et = np.fft.fftn(eta * phase, axes=(1, 2, 3, 4))
    px, py, pz, pt = _momenta(act)
    out = np.zeros_like(et)
    for it_ in range(Lt):
        for iz in range(Lz):
            for iy in range(Ly):
                for ix in range(Lx):
                    Dp = free_field_momentum_matrix(act, (px[ix], py[iy], pz[iz], pt[it_]))
                    rhs = et[:, it_, iz, iy, ix, :, :].reshape(4 * L5, 3)
                    out[:, it_, iz, iy, ix, :, :] = np.linalg.solve(Dp, rhs).reshape(L5, 4, 3)
    psi = np.fft.ifftn(out, axes=(1, 2, 3, 4))
    return psi / phase


# ---------------------------------------------------------------------------
# Sources.
# ---------------------------------------------------------------------------
def wall_inject(xi, act):
    """5D source from a 4D field xi[t][z][y][x][spin][col]: eta_0 = P- xi,
    eta_{L5-1} = P+ xi, zero elsewhere."""
    eta = np.zeros(act.shape5, dtype=np.complex128)
    eta[0] += _spin(PMINUS, xi)
    eta[act.L5 - 1] += _spin(PPLUS, xi)
    return eta


def point_source(act, x0=(0, 0, 0, 0), spin=0, colour=0):
    """Unit 4D point source at x0 = (x,y,z,t), wall-injected."""
    Lx, Ly, Lz, Lt = act.L
    xi = np.zeros((Lt, Lz, Ly, Lx, 4, 3), dtype=np.complex128)
    xi[x0[3], x0[2], x0[1], x0[0], spin, colour] = 1.0
    return wall_inject(xi, act)


_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, counter: int) -> int:
    """Output number ``counter`` (0-based) of SplitMix64 seeded with ``seed``.

    Steele, Lea, Flood, "Fast splittable pseudorandom number generators"
    (OOPSLA 2014): state_k = seed + (k+1)*0x9E3779B97F4A7C15 mod 2^64, then
    the variant-13 finaliser (shifts 30, 27, 31).
    """
    z = (seed + (counter + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def z2_noise(act, seed, rhs=0):
    """Complex Z2 4D noise xi = ((+-1) + i(+-1))/sqrt(2) per (site, spin, colour).

    Counter k = ((rhs*V4 + i4)*4 + spin)*3 + colour with
    i4 = ((t*Lz + z)*Ly + y)*Lx + x; bit 0 of the draw picks the sign of the
    real part, bit 1 that of the imaginary part.
    """
    Lx, Ly, Lz, Lt = act.L
    V4 = Lx * Ly * Lz * Lt
    n = V4 * 12
    # the same recurrence as splitmix64(), on uint64 arrays (wrapping arithmetic)
    k = np.arange(n, dtype=np.uint64) + np.uint64(rhs * n + 1)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + k * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    re = 1.0 - 2.0 * (z & np.uint64(1)).astype(np.float64)
    im = 1.0 - 2.0 * ((z >> np.uint64(1)) & np.uint64(1)).astype(np.float64)
    # 1/sqrt(2) correctly rounded (sqrt is correctly rounded; 1/np.sqrt(2) is not)
    xi = (re + 1j * im) * np.sqrt(0.5)
    return xi.reshape(Lt, Lz, Ly, Lx, 4, 3)


def z2_source(act, seed, rhs=0):
    return wall_inject(z2_noise(act, seed, rhs), act)


# ---------------------------------------------------------------------------
# Gauge transformations (for the covariance check).
# U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag ;  (G psi)_s(x) = g(x) psi_s(x)
# ---------------------------------------------------------------------------
def gauge_transform_links(U, g):
    out = np.empty_like(U)
    for mu in range(4):
        g_fwd = np.roll(g, -1, axis=_LINK_AXIS[mu])
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(g_fwd, -1, -2))
    return out


def gauge_transform_spinor(psi, g):
    return np.einsum("tzyxab,stzyxjb->stzyxja", g, psi)


# ---------------------------------------------------------------------------
# D psi at a few sampled 5D sites, summed term by term (for large lattices
# where a full application does not fit the CPU budget).
# ---------------------------------------------------------------------------
def dirac_at_sites(U, psi, act, sites):
    """(D psi) at sites [(s, t, z, y, x), ...]; returns an array [n][4][3].

    Expands D = M5 - 1/2 H M_phi site by site:
    (D psi)_s(x) = sum_s' [alpha d + beta P5]_{ss'} psi_s'(x)
                   - 1/2 sum_mu [(1-g_mu) U_mu(x) (M_phi psi)(x+mu)
                                 + (1+g_mu) U_mu(x-mu)^dag (M_phi psi)(x-mu)]_s
    """
    Lx, Ly, Lz, Lt = act.L
    L5 = act.L5
    alpha, beta = _coeffs(act)
    S_up, S_dn = fifth_matrices(L5, act.mq)
    A5p = alpha * np.eye(L5) + beta * S_dn
    A5m = alpha * np.eye(L5) + beta * S_up
    Php = act.b5 * np.eye(L5) + act.c5 * S_dn
    Phm = act.b5 * np.eye(L5) + act.c5 * S_up

    def mphi_col(t, z, y, x, s):
        col = psi[:, t, z, y, x]                                 # [L5][4][3]
        return Php[s] @ (PPLUS @ col.reshape(L5, 4, 3)).reshape(L5, 12) \
            + Phm[s] @ (PMINUS @ col.reshape(L5, 4, 3)).reshape(L5, 12)

    out = []
    for (s, t, z, y, x) in sites:
        col = psi[:, t, z, y, x].reshape(L5, 4, 3)
        local = (A5p[s] @ (PPLUS @ col).reshape(L5, 12) + A5m[s] @ (PMINUS @ col).reshape(L5, 12)).reshape(4, 3)
        h = np.zeros((4, 3), dtype=np.complex128)
        c = [x, y, z, t]
        L = [Lx, Ly, Lz, Lt]
        for mu in range(4):
            f = list(c)
            f[mu] = (c[mu] + 1) % L[mu]
            sgn_f = -1.0 if (mu == 3 and act.t_antiperiodic and c[mu] == L[mu] - 1) else 1.0
            b = list(c)
            b[mu] = (c[mu] - 1) % L[mu]
            sgn_b = -1.0 if (mu == 3 and act.t_antiperiodic and c[mu] == 0) else 1.0
            chi_f = sgn_f * mphi_col(f[3], f[2], f[1], f[0], s).reshape(4, 3)
            chi_b = sgn_b * mphi_col(b[3], b[2], b[1], b[0], s).reshape(4, 3)
            Uf = U[t, z, y, x, mu]
            Ub = U[b[3], b[2], b[1], b[0], mu]
            tf = chi_f @ Uf.T                                    # U chi per spin row
            tb = chi_b @ np.conj(Ub)                             # U^dag chi
            h += (IDENT4 - GAMMA[mu]) @ tf + (IDENT4 + GAMMA[mu]) @ tb
        out.append(local - 0.5 * h)
    return np.array(out)


# ---------------------------------------------------------------------------
# Feynman-Hellmann sequential propagator (paper, "Current State of the Art",
# Physics algorithms related: one extra propagator carries a current inserted
# at every time slice, giving all source-sink separations at the cost of one).
# Readings: the 4D quark field is read off the walls, q = P- psi_0 + P+
# psi_{L5-1} (the projection that matches the wall injection of a source; no
# Moebius 4D source factor); the current is a spin matrix Gamma, one of the 16
# products of gamma matrices, applied at every site; the sequential source is
# Gamma q, wall-injected like any 4D source; the sequential propagator solves
# D psi_FH = inject(Gamma q).
# ---------------------------------------------------------------------------
def gamma_product(mask: int) -> np.ndarray:
    """Gamma = g_x^b0 g_y^b1 g_z^b2 g_t^b3 for mask = b0 + 2 b1 + 4 b2 + 8 b3
    (mask 0 is the identity, mask 15 is gamma5)."""
    G = IDENT4.copy()
    for mu in range(4):
        if (mask >> mu) & 1:
            G = G @ GAMMA[mu]
    return G


def propagator_4d(psi, act):
    """4D field q[t][z][y][x][spin][col] = P- psi_0 + P+ psi_{L5-1}."""
    return _spin(PMINUS, psi[0]) + _spin(PPLUS, psi[act.L5 - 1])


def current_source(q, act, mask):
    """Sequential 5D source: the current Gamma applied to q at every site,
    wall-injected."""
    return wall_inject(_spin(gamma_product(mask), q), act)


def fh_solve(U, psi, act, mask, tol=1e-12):
    """psi_FH = D^{-1} inject(Gamma q(psi))."""
    return solve(U, current_source(propagator_4d(psi, act), act, mask), act, tol=tol)


def fh_operator(psi, act, mask):
    """J psi = inject(Gamma q(psi)): the 5D operator of the current
    insertion, so that D(lambda) = D + lambda J is the action with the
    current added; d/dlambda D(lambda)^{-1} eta = -D^{-1} J D^{-1} eta."""
    return current_source(propagator_4d(psi, act), act, mask)


# ---------------------------------------------------------------------------
# The physical 4D propagator of the Moebius action (Brower, Neff, Orginos,
# arXiv:1206.5214; the paper's "Physics algorithms related" paragraph needs it
# for the quark propagators its Feynman-Hellmann method combines).
# Readings: the antiquark field sits on the opposite walls to the quark field
# the read-out q = P- psi_0 + P+ psi_{L5-1} takes, so a 4D source xi enters
# as eta_0 = P+ xi, eta_{L5-1} = P- xi; and the Moebius operator
# D = (b5 D_W + 1) - (1 - c5 D_W) P5 is the Shamir-like operator
# (1 - c5 D_W)^-1 (b5 D_W + 1) - P5 multiplied by the 4D factor
# (1 - c5 D_W), which the source must carry: eta = (1 - c5 D_W) inject(xi).
# Then q = S xi with S = (D_eff^-1 - 1) / (1 - mq), D_eff the truncated
# overlap operator of the Moebius kernel (effective_propagator_4d).  With
# c5 = 0 (Shamir) the factor is the identity.
# ---------------------------------------------------------------------------
def wall_inject_physical(xi, act):
    """eta_0 = P+ xi, eta_{L5-1} = P- xi, zero elsewhere."""
    eta = np.zeros(act.shape5, dtype=np.complex128)
    eta[0] += _spin(PPLUS, xi)
    eta[act.L5 - 1] += _spin(PMINUS, xi)
    return eta


def dminus(U, psi, act):
    """(1 - c5 D_W) psi on every slice."""
    return psi - act.c5 * dirac_wilson(U, psi, act)


def physical_source(U, xi, act, mask=0):
    """5D source of the physical 4D propagator: (1 - c5 D_W) inject(Gamma xi),
    Gamma = gamma_product(mask) (mask 0: the identity)."""
    return dminus(U, wall_inject_physical(_spin(gamma_product(mask), xi), act), act)


def current_source_physical(U, q, act, mask):
    """Sequential source of the physical Feynman-Hellmann propagator: the
    current Gamma applied to the 4D propagator q at every site, entering as a
    physical source."""
    return physical_source(U, q, act, mask)


def fh_solve_physical(U, xi, act, mask, tol=1e-12):
    """(q, q_FH): the physical 4D propagator q = S xi and the sequential one
    q_FH = S Gamma q, each read off the walls of a 5D solve."""
    psi, _ = solve(U, physical_source(U, xi, act), act, tol=tol)
    q = propagator_4d(psi, act)
    psi2, _ = solve(U, current_source_physical(U, q, act, mask), act, tol=tol)
    return q, propagator_4d(psi2, act)


def effective_propagator_4d(U, act):
    """Dense 4D matrix S = (D_eff^-1 - 1) / (1 - mq) on a tiny lattice, with
    D_eff = (1 + mq)/2 + (1 - mq)/2 g5 eps(H_M), H_M = g5 (b5 + c5) D_W
    (2 + (b5 - c5) D_W)^-1 (Hermitian) and eps(H) = [(1+H)^L5 - (1-H)^L5]
    [(1+H)^L5 + (1-H)^L5]^-1, the polar approximation of sign(H) that L5
    slices realise.  Rows and columns index [t][z][y][x][spin][col]."""
    Lx, Ly, Lz, Lt = act.L
    shape4 = (Lt, Lz, Ly, Lx, 4, 3)
    n = int(np.prod(shape4))
    Dw = dense_matrix(lambda v: dirac_wilson(U, v[None], act)[0], shape4)
    g5 = np.kron(np.eye(n // 12), np.kron(GAMMA5, np.eye(3)))
    I = np.eye(n)
    HM = g5 @ ((act.b5 + act.c5) * Dw) @ np.linalg.inv(2.0 * I + (act.b5 - act.c5) * Dw)
    A = np.linalg.matrix_power(I + HM, act.L5)
    B = np.linalg.matrix_power(I - HM, act.L5)
    E = (A - B) @ np.linalg.inv(A + B)
    Deff = 0.5 * (1.0 + act.mq) * I + 0.5 * (1.0 - act.mq) * g5 @ E
    return (np.linalg.inv(Deff) - I) / (1.0 - act.mq)
