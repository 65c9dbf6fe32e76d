"""Host-side arithmetic the kernels rely on, checked on the CPU.

Site coordinates divide checkerboard indices by Lx/2, Ly and Lz with a
32-bit multiply-high: q = (n * m) >> 32, m = floor(2^32 / d) + 1.  With
e = m*d - 2^32 in (0, d], n*m/2^32 = n/d + n*e/(d*2^32), whose excess stays
below 1/d (so the floor is unchanged) whenever n*d < 2^32 — the bound the
library enforces when it validates an action.  Brute force over the worst
cases (n just below a multiple of d, n at the bound) for every divisor a
lattice extent can take."""
import random


def _magic(d):
    return 0 if d <= 1 else (1 << 32) // d + 1


def test_fastdiv_exact_below_bound():
    rng = random.Random(5)
    for d in list(range(1, 1025)):
        m = _magic(d)
        lim = ((1 << 32) - 1) // d  # largest n with n*d < 2^32
        ns = {0, 1, d - 1, d, d + 1, lim, lim - 1, (lim // d) * d - 1, (lim // d) * d}
        ns.update(rng.randrange(lim + 1) for _ in range(200))
        for n in ns:
            if n < 0 or n * d >= 1 << 32:
                continue
            q = n if m == 0 else (n * m) >> 32
            assert q == n // d, (n, d)


def test_fastdiv_bound_is_needed():
    # beyond the bound the multiply-high can overshoot: the check is not vacuous
    d = 2
    m = _magic(d)
    n = (1 << 32) - 1
    assert n * d >= 1 << 32 and (n * m) >> 32 != n // d


def test_traversal_overrides_are_clamped(monkeypatch):
    """The stencil's workgroup traversal after the MDWF_BT / MDWF_YB
    overrides: negative or non-dividing values fall back to the linear order
    (Bt = 0) and one band, so a mistyped override can never produce
    out-of-range site indices (host-side query, no GPU)."""
    from paper_1810_01609_amd import mdwf as M

    act = M.Action.make((32, 32, 32, 64), 12, mq=0.005)
    monkeypatch.delenv("MDWF_BT", raising=False)
    monkeypatch.delenv("MDWF_YB", raising=False)
    assert M.query_traversal(act, "f16", 12) == (2, 8)  # L5 <= 12: 4-row bands, Bt = 2
    act16 = M.Action.make((24, 24, 24, 64), 16, mq=0.01)
    bt, yb = M.query_traversal(act16, "f16", 1)
    assert yb == 1 and bt in (2, 4, 8) and 64 % bt == 0
    for bt_env, yb_env, want in (("-3", "-2", (2, 8)),     # ignored: defaults stay
                                 ("0", "1", (0, 1)),       # linear order, one band
                                 ("3", "8", (0, 8)),       # 3 does not divide Lt = 64
                                 ("4", "5", (4, 1)),       # 5 does not divide Ly = 32
                                 ("8", "16", (8, 16)),     # 2-row bands: 16 x 2 = 32 sites, two workgroups
                                 ("2", "64", (2, 1))):     # 64 bands of half a row: not whole workgroups
        monkeypatch.setenv("MDWF_BT", bt_env)
        monkeypatch.setenv("MDWF_YB", yb_env)
        assert M.query_traversal(act, "f16", 12) == want, (bt_env, yb_env)
    with __import__("pytest").raises(M.MDWFError):
        M.query_traversal(act, "f16", 12, cb_log2=9)
