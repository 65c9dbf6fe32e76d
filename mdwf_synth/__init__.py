"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only *draws data*: SU(3) gauge links, random spinor fields, random
gauge transformations and request traces.  It holds none of the solver's
arithmetic (no Dirac operator, no projection, no 5th-dimension algebra, no
source wall-injection), so that the oracle and the HIP path can both consume
the same inputs without sharing any of the method.

Layouts (user / ABI layouts, identical on both sides):

* gauge  : complex128 ``[t][z][y][x][mu][row][col]``, mu = 0,1,2,3 <-> x,y,z,t
* spinor : complex128 ``[s][t][z][y][x][spin][colour]`` (one right-hand side)

The paper gives neither its ensembles nor a generator; links here follow the
recipe ``U = exp(i*eps*H)`` with ``H`` a Gaussian traceless Hermitian matrix,
then re-unitarised (Gram-Schmidt on rows 0-1, row 2 = conj(row0 x row1)).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gauge_field",
    "random_su3",
    "random_spinor",
    "random_gauge_transform",
    "poisson_trace",
    "CONFIGS",
]


def _reunitarise(U: np.ndarray) -> np.ndarray:
    """Project a stack of near-unitary 3x3 matrices onto SU(3).

    Rows 0 and 1 are orthonormalised by Gram-Schmidt, row 2 is the complex
    conjugate of their cross product, which fixes det = +1.
    """
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def random_su3(shape, eps: float, rng: np.random.Generator) -> np.ndarray:
    """SU(3) matrices exp(i*eps*H), H Gaussian traceless Hermitian, shape + (3,3)."""
    G = rng.standard_normal(tuple(shape) + (3, 3, 2))
    A = G[..., 0] + 1j * G[..., 1]
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1)[..., None, None] / 3.0
    H = H - tr * np.eye(3)
    w, V = np.linalg.eigh(H)
    U = (V * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(V, -1, -2))
    return _reunitarise(U)


def gauge_field(L, eps: float, seed: int) -> np.ndarray:
    """Synthetic gauge configuration, complex128 [t][z][y][x][mu][3][3].

    ``L = (Lx, Ly, Lz, Lt)``.  ``eps = 0`` gives the free field U = 1.
    """
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(random_su3((Lt, Lz, Ly, Lx, 4), eps, rng))


def unit_gauge(L) -> np.ndarray:
    """Free field: every link is the identity."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def random_gauge_transform(L, seed: int, eps: float = 1.0) -> np.ndarray:
    """One SU(3) matrix g(x) per 4D site, complex128 [t][z][y][x][3][3]."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(random_su3((Lt, Lz, Ly, Lx), eps, rng))


def random_spinor(L, L5: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Gaussian complex 5D spinor field, complex128 [(rhs)][s][t][z][y][x][4][3]."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    rng = np.random.default_rng(seed)
    shape = (int(L5), Lt, Lz, Ly, Lx, 4, 3)
    if nrhs is not None:
        shape = (int(nrhs),) + shape
    G = rng.standard_normal(shape + (2,))
    return np.ascontiguousarray(G[..., 0] + 1j * G[..., 1])


def poisson_trace(n_requests: int, rate_hz: float, seed: int, volumes, l5s, mq_range, nsrc_range):
    """A finite request trace with Poisson arrivals (exponential gaps).

    Returns a list of dicts ``{id, t_arrival, volume, L5, mq, nsrc}``; every
    choice is uniform over the given sets / ranges.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        out.append(
            dict(
                id=i,
                t_arrival=float(t[i]),
                volume=tuple(volumes[int(rng.integers(len(volumes)))]),
                L5=int(l5s[int(rng.integers(len(l5s)))]),
                mq=float(rng.uniform(*mq_range)),
                nsrc=int(rng.integers(nsrc_range[0], nsrc_range[1] + 1)),
            )
        )
    return out


# The benchmark workloads: lattice (Lx,Ly,Lz,Lt), L5, Moebius parameters,
# quark mass, link smearing eps and seed, source choice.
CONFIGS = {
    "c1": dict(L=(4, 4, 4, 8), L5=8, b5=1.5, c5=0.5, M5=1.3, mq=0.05, eps=0.3, seed=1,
               source="point", z2_seed=None),
    "c2": dict(L=(16, 16, 16, 32), L5=12, b5=1.5, c5=0.5, M5=1.3, mq=0.02, eps=0.2, seed=2,
               source="z2", z2_seed=1002),
    "c3": dict(L=(24, 24, 24, 64), L5=16, b5=1.5, c5=0.5, M5=1.3, mq=0.01, eps=0.15, seed=3,
               source="z2", z2_seed=1003),
    "c4": dict(L=(32, 32, 32, 64), L5=12, b5=1.5, c5=0.5, M5=1.3, mq=0.005, eps=0.15, seed=4,
               source="point12", z2_seed=None),
}
