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


def make_case(L, L5, mq, eps, seed, tap=1):
    from paper_1810_01609_amd import mdwf as M
    import oracle as O

    U = S.gauge_field(L, eps, seed) if eps > 0 else S.unit_gauge(L)
    act = M.Action.make(L, L5, 1.5, 0.5, 1.3, mq, tap)
    oact = O.Action(L, L5, 1.5, 0.5, 1.3, mq, t_antiperiodic=bool(tap))
    return U, act, oact
