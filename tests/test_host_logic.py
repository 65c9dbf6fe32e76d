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
