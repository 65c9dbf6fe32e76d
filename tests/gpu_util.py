"""Helpers shared by the GPU tests (no tests here)."""
import sys

import numpy as np

import mdwf_synth as S


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def empty_like_dev(shape):
    import torch

    return torch.zeros(shape, dtype=torch.complex128, device="cuda")


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def errors(got, ref):
    """(norm-wise, element-wise) relative error of got against ref:
    |got - ref| / |ref| and max|got - ref| / max|ref|."""
    d = np.abs(got - ref)
    mref = np.abs(ref).max()
    return rel(got, ref), (d.max() / mref if mref > 0 else d.max())


def check(got, ref, tol, what):
    """Assert both the norm-wise and the element-wise relative error are
    within tol, and log the measured values."""
    en, ee = errors(got, ref)
    log(f"   {what}: norm-wise {en:.2e} element-wise {ee:.2e} (bar {tol:.0e})")
    assert en <= tol and ee <= tol, (what, en, ee, tol)
    return en, ee


def make_case(L, L5, mq, eps, seed, tap=1):
    from paper_1810_01609_amd import mdwf as M
    import oracle as O

    U = S.gauge_field(L, eps, seed) if eps > 0 else S.unit_gauge(L)
    act = M.Action.make(L, L5, 1.5, 0.5, 1.3, mq, tap)
    oact = O.Action(L, L5, 1.5, 0.5, 1.3, mq, t_antiperiodic=bool(tap))
    return U, act, oact
