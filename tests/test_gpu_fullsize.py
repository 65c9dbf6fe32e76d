"""Parity at the benchmark sizes, in the launch configuration the benchmark
uses, on sampled outputs the oracle computes site by site
(``oracle.dirac_at_sites``): the full operator D on C2/C3/C4 lattices in
every precision, and the FP64 full residual eta - D psi of GPU solves.

Residual bar: |eta - D psi| / |eta| < 1e-8 norm-wise and max|eta - D psi| <
1e-8 max|eta| element-wise, with D the FP64 oracle's (the solves stop at
1e-10 on the normal equations; the full residual is ~1e-10 relative)."""
import numpy as np
import pytest

import mdwf_synth as S
import oracle as O
from gpu_util import check, empty_like_dev, log, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 8e-3, "bf16": 6e-2, "i16": 1e-3}


def _sites(L, L5, n, seed):
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz, Lt = L
    pts = [(0, 0, 0, 0, 0), (L5 - 1, Lt - 1, Lz - 1, Ly - 1, Lx - 1), (0, Lt - 1, 0, 0, 1), (L5 - 1, 0, 1, 0, 0)]
    for _ in range(n - len(pts)):
        pts.append((int(rng.integers(L5)), int(rng.integers(Lt)), int(rng.integers(Lz)), int(rng.integers(Ly)),
                    int(rng.integers(Lx))))
    return pts


@pytest.fixture(scope="module")
def ctx():
    from paper_1810_01609_amd import mdwf as M

    c = M.Context(0)
    yield c
    c.close()


def _cfg(name):
    from paper_1810_01609_amd import mdwf as M

    c = S.CONFIGS[name]
    act = M.Action.make(c["L"], c["L5"], c["b5"], c["c5"], c["M5"], c["mq"])
    oact = O.Action(c["L"], c["L5"], c["b5"], c["c5"], c["M5"], c["mq"])
    U = S.gauge_field(c["L"], c["eps"], c["seed"])
    return c, act, oact, U


@pytest.mark.parametrize("name,precs", [("c2", ("f64", "f32", "f16", "bf16", "i16")), ("c3", ("f32", "f16", "bf16", "i16")),
                                        ("c4", ("f32", "f16"))])
def test_dirac_sampled_full_size(ctx, name, precs):
    from paper_1810_01609_amd import mdwf as M

    c, act, oact, U = _gauge(name)
    log(f"[full] D on {name} {c['L']} L5={c['L5']}")
    g = ctx.gauge_load(c["L"], U, precs=("f64",) + tuple(p for p in precs if p != "f64"))
    x = S.random_spinor(c["L"], c["L5"], 31)
    sites = _sites(c["L"], c["L5"], 256, 7)
    expect = O.dirac_at_sites(U, x, oact, sites)
    xd = to_dev(x)
    out = empty_like_dev(x.shape)
    for p in precs:
        ctx.dslash(g, act, M.OP_D, p, xd, out)
        got = to_host(out)
        sel = np.array([got[s] for s in sites])
        check(sel, expect, TOL[p], f"D {name} {p} at {len(sites)} sampled sites")
    del xd, out
    g.free()


_U = {}


def _gauge(name):
    if name not in _U:
        _U.clear()
        _U[name] = _cfg(name)
    return _U[name]


# (config, inner precision, right-hand sides, oracle check): "full" applies the
# oracle's D to the whole GPU solution (c2: ~15-30 s of NumPy), an integer
# applies it at that many sampled sites per right-hand side (c3, c4: a full
# oracle D there costs minutes per field)
SOLVES = [("c2", "f32", 1, "full"), ("c2", "f64", 1, "full"), ("c3", "f16", 1, 4096), ("c3", "bf16", 1, 2048),
          ("c3", "i16", 1, 2048), ("c4", "f16", 12, 384), ("c4", "f32", 12, 384)]


@pytest.mark.parametrize("name,inner,nrhs,verify", SOLVES)
def test_solve_oracle_residual_full_size(ctx, name, inner, nrhs, verify):
    """The benchmark solves (c4: all 12 spin-colour point sources fused in one
    solve), each result verified with the FP64 oracle's D: the relative
    residual |eta - D psi| / |eta| must stay below 1e-8 norm-wise, and
    max|eta - D psi| below 1e-8 max|eta| element-wise."""
    import torch

    from paper_1810_01609_amd import mdwf as M

    c, act, oact, U = _gauge(name)
    torch.cuda.empty_cache()  # c4 with 12 RHS needs ~270 GB of the 288
    ctx.trim()  # and the previous solve's cached state goes too
    g = ctx.gauge_load(c["L"], U, precs=("f64", inner))
    eta = torch.zeros((nrhs,) + act.spinor_shape(), dtype=torch.complex128, device="cuda")
    for r in range(nrhs):
        if c["source"] == "z2":
            ctx.source_z2(act, c["z2_seed"], r, eta[r])
        else:
            ctx.source_point(act, (0, 0, 0, 0), r // 3, r % 3, eta[r])
    psi = torch.zeros_like(eta)
    log(f"[full] solve {name} {inner} nrhs={nrhs}")
    stats = ctx.solve(g, act, M.CGOpts.make(tol=1e-10, inner=inner), eta, psi, nrhs=nrhs)
    for r in range(nrhs):
        st = stats[r]
        log(f"[full] solve {name} {inner} rhs {r}: iters={st['iters']} updates={st['reliable_updates']} "
            f"res_normal={st['rel_res_normal']:.2e} res_full(gpu fp64)={st['rel_res_full']:.2e} {st['seconds']:.2f}s")
        assert st["converged"] == 1 and st["rel_res_normal"] <= 1e-10
        assert st["rel_res_full"] < 1e-8
        e = to_host(eta[r])
        p = to_host(psi[r])
        if verify == "full":
            res = e - O.dirac(U, p, oact)
            rn = np.linalg.norm(res) / np.linalg.norm(e)
            re = np.abs(res).max() / np.abs(e).max()
            log(f"   oracle residual (whole field): norm-wise {rn:.2e} element-wise {re:.2e}")
        else:
            sites = _sites(c["L"], c["L5"], verify, 11 + r)
            # the source's own sites (point sources: the wall slices at the origin)
            sites += [(c["L5"] - 1, 0, 0, 0, 0), (0, 0, 0, 0, 0), (0, 0, 0, 0, 1), (c["L5"] - 1, 0, 0, 1, 0)]
            es = np.array([e[s] for s in sites])
            res = es - O.dirac_at_sites(U, p, oact, sites)
            # norm-wise over the sample, scaled to the whole field: the sampled
            # |res|^2 times (field sites / sampled sites) against |eta|^2
            frac = len(sites) / (np.prod(c["L"]) * c["L5"])
            rn = np.sqrt(np.sum(np.abs(res) ** 2) / frac) / np.linalg.norm(e)
            re = np.abs(res).max() / np.abs(e).max()
            log(f"   oracle residual ({len(sites)} sampled sites): norm-wise estimate {rn:.2e} element-wise {re:.2e}")
        assert rn < 1e-8 and re < 1e-8, (rn, re)
        del e, p
    del eta, psi
    g.free()
