"""Benchmark: Moebius domain-wall propagator solves on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4]

Default workload (c4, the largest configuration, quoted in RHS/s): lattice
32^3 x 64, L5 = 12, b5 = 1.5, c5 = 0.5, M5 = 1.3, m_q = 0.005, links
exp(i 0.15 H) seed 4, the 12 spin-colour point sources at the origin.  One
step is one pass of the whole solve path over that batch: the 12 sources
generated on the device, even-odd source preparation, one fused 12-RHS
mixed-precision CG (FP16 storage with per-site scales, FP32 arithmetic, FP64
reliable updates and reductions) to |b - A x| <= 1e-10 |b| for every RHS,
reconstruction of the odd half and the FP64 full-5D residual check.  The
gauge field is resident in HBM before timing starts.  `value` is solved
right-hand sides per second over the timed steps; the JSON line also carries
the per-step latency percentiles, the plain FP64 single-RHS solver on the
same input, the fused stencil kernel's roofline (algorithmic bytes per launch
/ its average HIP-event duration, the events riding in the kernel dispatches
of one CG iteration in 13), the library's STREAM-style copy rate measured in
the same run, and the CPU oracle's rate on a bounded sample of the workload.
Other workloads (c1, c2, c3, c5 serving) and modes (--dslash-only, --fh,
--split) are selected by flags.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dslash.hip", "dev_common.h"):
        with open(os.path.join(ROOT, "paper_1810_01609_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch of the fused stencil kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"dslash_{workload}_hbm_traffic.json")
    if not os.path.exists(path):
        return None, "no counter summary"
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sha") != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    return d.get("traffic_bytes_per_launch"), d.get("note", "")


def cpu_baseline(cfg, gpu_iters_f64: int):
    """The oracle as it stands, timed on a bounded sample of the workload.

    Each of the oracle's building blocks is applied once to a field (one 4D
    hop H, one M5^-1, one M_phi: ~10-30 s of CPU work in all).  Up to 2M 5D
    sites the field covers the whole lattice; beyond, a slab of the lattice
    (the full Lx, Ly, Lz and the fewest time slices that still hold ~1.5M 5D
    sites, with the workload's L5) stands in for it, and the times are scaled
    by the volume ratio (the oracle's cost per site does not depend on the
    volume: every step is a whole-array NumPy operation).  The solve time is
    then composed from how often the oracle's even-odd CGNR calls them: per
    iteration 4 hops, 4 M5^-1 and 4 M_phi (M^ and M^+), plus setup (source
    preparation and b = M^+ eta^: 3 hops, 4 M5^-1, 3 M_phi), times the FP64
    iteration count of the same solve on the GPU.  One right-hand side.
    """
    import mdwf_synth as S
    import oracle as O

    L = list(cfg["L"])
    L5 = cfg["L5"]
    v5 = L[0] * L[1] * L[2] * L[3] * L5
    scale = 1.0
    if v5 > 2_000_000:
        lt = max(2, int(1.5e6 / (L[0] * L[1] * L[2] * L5)) // 2 * 2)
        scale = L[3] / lt
        L[3] = lt
    act = O.Action(tuple(L), L5, cfg["b5"], cfg["c5"], cfg["M5"], cfg["mq"])
    U = S.gauge_field(tuple(L), cfg["eps"], cfg["seed"])
    x = S.random_spinor(tuple(L), L5, 7)
    t = {}
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):  # one thread, whatever BLAS NumPy links
        for name, fn in (("hop", lambda: O.hop(U, x, act)), ("m5_inv", lambda: O.m5_inv(x, act)),
                         ("m_phi", lambda: O.m_phi(x, act))):
            t0 = time.perf_counter()
            fn()
            t[name] = (time.perf_counter() - t0) * scale
    per_iter = 4 * t["hop"] + 4 * t["m5_inv"] + 4 * t["m_phi"]
    setup = 3 * t["hop"] + 4 * t["m5_inv"] + 3 * t["m_phi"]
    t_solve = setup + per_iter * gpu_iters_f64
    where = (f"the full {cfg['L'][0]}^3x{cfg['L'][3]} L5={L5} lattice" if scale == 1.0 else
             f"a {L[0]}x{L[1]}x{L[2]}x{L[3]} L5={L5} slab of the {cfg['L'][0]}^3x{cfg['L'][3]} lattice, "
             f"times scaled by {scale:g} to the whole volume")
    return {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle hop, M5^-1 and M_phi each applied once (NumPy FP64, one thread) on {where}; solve time "
                   f"(one RHS) composed as setup + {gpu_iters_f64} CGNR iterations x (4 hop + 4 M5^-1 + 4 M_phi), "
                   f"the oracle's own call counts, with the FP64 iteration count of the same solve"),
        "estimate": scale != 1.0,
        "component_seconds": t,
        "seconds_per_iteration": per_iter,
        "host_cpus": os.cpu_count(),
        "cpu_model": _cpu_model(),
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def progress(msg):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stats_flops(stats, nrhs):
    """Modelled flops of the timed solves (the library's per-iteration count
    times the iterations of each RHS)."""
    return sum(s["flops"] for s in stats)


def fh_bench(args):
    """Feynman-Hellmann sequential propagators: per step, the Z2 source, the
    propagator solve, the 4D read-out, the current source (axial g_x g_y g_t,
    mask 11) and the sequential solve, all on the device."""
    import torch

    import mdwf_synth as S
    from paper_1810_01609_amd import mdwf as M

    cfg = S.CONFIGS[args.workload]
    inner = args.inner or ("f16" if args.workload in ("c3", "c4") else "f32")
    L, L5 = cfg["L"], cfg["L5"]
    act = M.Action.make(L, L5, cfg["b5"], cfg["c5"], cfg["M5"], cfg["mq"])
    U = S.gauge_field(L, cfg["eps"], cfg["seed"])
    ctx = M.Context(0)
    g = ctx.gauge_load(L, U, precs=("f64", inner))
    del U
    eta = torch.zeros(act.spinor_shape(), dtype=torch.complex128, device="cuda")
    psi = torch.zeros_like(eta)
    q = torch.zeros(act.spinor_shape()[1:], dtype=torch.complex128, device="cuda")
    eta2 = torch.zeros_like(eta)
    fh = torch.zeros_like(eta)
    opts = M.CGOpts.make(tol=1e-10, inner=inner)

    xi = torch.zeros_like(q)

    def step():
        seed = cfg["z2_seed"] if cfg["source"] == "z2" else 1
        ctx.source_z2(act, seed, 0, eta)
        if args.physical:
            # the 4D noise itself (reading the walls back inverts the injection),
            # then the physical source (1 - c5 D_W) inject(xi)
            ctx.propagator_4d(act, eta, xi)
            ctx.source_physical(g, act, xi, eta)
        s1 = ctx.solve(g, act, opts, eta, psi)[0]
        ctx.propagator_4d(act, psi, q)
        if args.physical:
            ctx.source_physical(g, act, q, eta2, gamma_mask=11)
        else:
            ctx.current_source(act, 11, q, eta2)
        s2 = ctx.solve(g, act, opts, eta2, fh)[0]
        return s1, s2

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ok = all(a["converged"] == 1 and b["converged"] == 1 for a, b in stats)
    g.free()
    ctx.close()
    line = {
        "metric": "Feynman-Hellmann propagator pairs/s (propagator + sequential solve, each to rel-res 1e-10)",
        "value": args.steps / el if ok else 0.0, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if inner == "f64" else "f32", "data": "synthetic",
        "config": {"workload": (f"{args.workload} Feynman-Hellmann: Z2 source, axial current g_x g_y g_t, {inner} inner"
                                + (", physical 4D propagators (Moebius source factor)" if args.physical else ""))},
        "iters": [stats[-1][0]["iters"], stats[-1][1]["iters"]],
        "rel_res_full": [stats[-1][0]["rel_res_full"], stats[-1][1]["rel_res_full"]],
    }
    print(json.dumps(line), flush=True)


def split_bench(args):
    """One rank's share of a domain-decomposed hop: the workload's lattice cut
    in two along y, z and t (the 2x2x2 split of eight GPUs), the local block
    computed with its faces packed, the interior hop, and the exterior update
    from the faces (the lattice is its own neighbour: the exchange over xGMI is
    what one GPU cannot show, so its time is projected from the face bytes)."""
    import torch

    import mdwf_synth as S
    from paper_1810_01609_amd import mdwf as M

    cfg = S.CONFIGS[args.workload]
    Lg, L5 = cfg["L"], cfg["L5"]
    mask = 0b1110
    L = tuple(n // 2 if (mask >> m) & 1 else n for m, n in enumerate(Lg))
    act = M.Action.make(L, L5, cfg["b5"], cfg["c5"], cfg["M5"], cfg["mq"])
    ctx = M.Context(0)
    U = S.gauge_field(L, cfg["eps"], cfg["seed"])
    precs = args.precs.split(",")
    g = ctx.gauge_load(L, U, precs=tuple(dict.fromkeys(["f64"] + precs)))
    del U
    x = torch.zeros(act.spinor_shape(), dtype=torch.complex128, device="cuda")
    ctx.source_z2(act, 7, 0, x)
    y = torch.zeros_like(x)
    vh = L[0] * L[1] * L[2] * L[3] // 2
    out = {}
    for p in precs:
        rb = 8 if p == "f64" else 4
        face = {m: 2 * (vh * 2 // L[m] // 2) * L5 * 12 * rb for m in range(4) if (mask >> m) & 1}
        res = {}
        for name, m in (("plain", 0), ("split", mask)):
            for _ in range(2):
                ctx.hop_split(g, act, p, m, x, y)
            ctx.profile_enable(True)
            ctx.profile_reset()
            ph = [0.0, 0.0, 0.0]
            for _ in range(args.steps):
                t = ctx.hop_split(g, act, p, m, x, y, timed=True)
                ph = [a + b for a, b in zip(ph, t)]
            d = ctx.profile_read(M.PROF_DSLASH_F64 if p == "f64" else M.PROF_DSLASH_INNER)
            ctx.profile_enable(False)
            ph = [v / args.steps for v in ph]
            res[name] = {"pack_ms": ph[0], "hop_ms": ph[1], "exterior_ms": ph[2],
                         "hop_GB_per_s": d["bytes"] / (d["ms"] * 1e-3) / 1e9}
        link_gbs = 153.0
        res["face_bytes_per_peer"] = face
        res["xgmi_ms_per_peer_link"] = {m: b / (link_gbs * 1e9) * 1e3 for m, b in face.items()}
        res["split_total_ms"] = res["split"]["pack_ms"] + res["split"]["hop_ms"] + res["split"]["exterior_ms"]
        res["overhead_vs_plain"] = res["split_total_ms"] / res["plain"]["hop_ms"] - 1.0
        out[p] = res
    g.free()
    ctx.close()
    print(json.dumps({"workload": f"{args.workload} split 2x2x2 in (y, z, t): one rank's block",
                      "local_lattice": list(L), "L5": L5, "split_mask": mask, "steps": args.steps,
                      "xgmi_link_GB_per_s": 153.0, "hop": out}), flush=True)


def serve_bench(args):
    """c5: a Poisson stream of solves served with continuous batching in the
    mixed precision, then (with --fifo-baseline) the same trace served by the
    plain baseline: first in, first out, one right-hand side at a time, FP64
    CG.  Both report p50/p99 latency and solved right-hand sides per second."""
    import mdwf_synth as S
    from paper_1810_01609_amd.serve import (GPUBackend, Request, merge_chunks, percentiles, serve_fifo, serve_gpu,
                                            split_requests)

    vols = [(8, 8, 8, 16), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]
    trace = S.poisson_trace(args.requests, args.rate, 5, vols, [8, 12, 16], (0.005, 0.05), (1, 12))

    def make_reqs():
        return [Request(id=d["id"], t_arrival=d["t_arrival"], volume=d["volume"], L5=d["L5"], mq=d["mq"],
                        nsrc=d["nsrc"], seed=100000 + d["id"]) for d in trace]

    import torch

    def report(kind):
        def f(k, n, t, used=None):
            free, total = torch.cuda.mem_get_info()
            adm = "" if used is None else f", admitted {used / 1e9:.0f} GB"
            progress(f"{kind}: {k}/{n} done after {t:.0f} s{adm}; device free {free / 1e9:.0f} of "
                     f"{total / 1e9:.0f} GB, torch allocated {torch.cuda.memory_allocated() / 1e9:.0f} GB, "
                     f"reserved {torch.cuda.memory_reserved() / 1e9:.0f} GB")
        return f

    inner = args.inner or "f16"
    seeds = {v: 11 + i for i, v in enumerate(vols)}
    be = GPUBackend(vols, gauge_eps=0.2, gauge_seeds=seeds, inner=inner)
    budget = int(args.hbm_budget_gb * 1e9) - be.resident_bytes
    sched, _, wall = serve_gpu(split_requests(make_reqs(), args.max_rhs), be, budget,
                               iters_per_step=args.iters_per_step, max_slots_per_lane=args.max_slots,
                               progress=report("continuous batching"))
    be.close()
    done = merge_chunks(sched.done)
    nrhs = sum(r.nsrc for r in done)
    ok = all(s.get("converged") == 1 for r in done for s in r.stats)
    p = percentiles(done)
    base = None
    if args.fifo_baseline:
        be64 = GPUBackend(vols, gauge_eps=0.2, gauge_seeds=seeds, inner="f64")
        kf = len(trace) if args.fifo_requests is None else min(args.fifo_requests, len(trace))
        fdone, _, fwall = serve_fifo(make_reqs()[:kf], be64, progress=report("FP64 FIFO"))
        be64.close()
        fn = sum(r.nsrc for r in fdone)
        fok = all(s.get("converged") == 1 for r in fdone for s in r.stats)
        base = {"solves_per_s": fn / fwall if fok else 0.0, "latency_ms": percentiles(fdone), "wall_s": fwall,
                "rhs_completed": fn, "converged_all": fok, "requests": kf,
                "kind": (f"FP64 CG, one right-hand side at a time, requests first in first out; the first {kf} "
                         f"requests of the same trace at their arrival times")}
    line = {
        "metric": "MDWF CG solves/s at rel-res 1e-10; Dslash HBM GB/s; p50/p99 solve latency",
        "value": nrhs / wall if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1, "steps": len(done), "warmup": 0, "ms_per_step": 1e3 * wall / max(len(done), 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64" if inner == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": (f"c5: Poisson stream of {args.requests} requests at {args.rate}/s (trace seed 5) over "
                                f"volumes {vols}, L5 in {{8,12,16}}, mq U[0.005,0.05], 1-12 Z2 sources, "
                                f"chunks of <= {args.max_rhs} RHS, {inner} inner, continuous batching"),
                   "budget_gb": budget / 1e9},
        "latency_ms": p,
        "rhs_completed": nrhs, "wall_s": wall, "peak_hbm_gb": sched.peak_used / 1e9, "converged_all": ok,
        "fifo_fp64_baseline": base,
    }
    print(json.dumps(line), flush=True)


def dslash_bench(args):
    """Stencil throughput: M^+M^ (the four fused launches of one CG
    iteration, without the BLAS) applied repeatedly in each precision."""
    import torch

    import mdwf_synth as S
    from paper_1810_01609_amd import mdwf as M

    cfg = S.CONFIGS[args.workload]
    L, L5 = cfg["L"], cfg["L5"]
    nrhs = args.nrhs
    act = M.Action.make(L, L5, cfg["b5"], cfg["c5"], cfg["M5"], cfg["mq"])
    ctx = M.Context(0)
    ctx.tune_mode(1 if args.tune else 0)
    U = S.gauge_field(L, cfg["eps"], cfg["seed"])
    precs = args.precs.split(",")
    g = ctx.gauge_load(L, U, precs=tuple(dict.fromkeys(["f64"] + precs)))
    del U
    x = torch.zeros((nrhs,) + act.spinor_shape(), dtype=torch.complex128, device="cuda")
    for r in range(nrhs):
        ctx.source_z2(act, 7, r, x[r])
    y = torch.zeros_like(x)
    out = {}
    op = {"normal": M.OP_NORMAL, "hop": M.OP_HOP_EO}[args.op]
    for p in precs:
        cls = M.PROF_DSLASH_F64 if p == "f64" else M.PROF_DSLASH_INNER
        for _ in range(2):
            ctx.dslash(g, act, op, p, x, y, nrhs=nrhs)
        ctx.profile_enable(True)
        ctx.profile_reset()
        for _ in range(args.steps):
            ctx.dslash(g, act, op, p, x, y, nrhs=nrhs)
        d = ctx.profile_read(cls)
        ctx.profile_enable(False)
        avg = d["ms"] / d["launches"]
        gbs = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        out[p] = {"GB_per_s": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS, "avg_launch_ms": avg,
                  "bytes_per_launch": d["bytes"] / d["launches"], "launches": d["launches"]}
    if args.tune_save:
        ctx.tune_save(args.tune_save)
    g.free()
    del x, y
    torch.cuda.empty_cache()
    # achievable HBM bandwidth for context: the library's copy kernel, 4 GiB
    a = torch.ones(1 << 28, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    copy_gbs = ctx.copy_bandwidth(a, b, reps=10)
    ctx.close()
    print(json.dumps({"workload": args.workload, "lattice": list(L), "L5": L5, "nrhs": nrhs,
                      "op": {"normal": "M^+M^ (4 fused stencil launches)", "hop": "H_eo (plain 4D hop)"}[args.op],
                      "tuned": bool(args.tune), "dslash": out,
                      "copy_kernel_GB_per_s": copy_gbs}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--inner", default=None, help="inner precision (default: f32 for c1/c2, f16 for c3/c4)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sequential", action="store_true",
                    help="solve the workload's right-hand sides one after another instead of fused (c4)")
    ap.add_argument("--skip-f64", action="store_true", help="skip the plain FP64 reference solve (profiling runs)")
    ap.add_argument("--requests", type=int, default=200, help="c5: requests in the trace")
    ap.add_argument("--fifo-baseline", action="store_true",
                    help="c5: also serve the trace first-in-first-out, one RHS at a time, in FP64")
    ap.add_argument("--fifo-requests", type=int, default=None,
                    help="c5: serve only the first K requests of the trace in the FIFO baseline (default: all)")
    ap.add_argument("--rate", type=float, default=20.0, help="c5: mean arrivals per second")
    ap.add_argument("--max-rhs", type=int, default=4, help="c5: largest chunk of sources admitted at once")
    ap.add_argument("--max-slots", type=int, default=16, help="c5: largest fused batch per lane")
    ap.add_argument("--iters-per-step", type=int, default=25, help="c5: iterations between batch changes")
    ap.add_argument("--hbm-budget-gb", type=float, default=float(os.environ.get("MDWF_HBM_BUDGET_GB", 240.0)),
                    help="c5: device memory for jobs (default: MDWF_HBM_BUDGET_GB, else 240)")
    ap.add_argument("--dslash-only", action="store_true", help="stencil throughput of M^+M^ per precision")
    ap.add_argument("--precs", default="f64,f32,f16,bf16")
    ap.add_argument("--op", default="normal", choices=("normal", "hop"),
                    help="dslash-only: the normal operator's four launches, or the plain 4D hop")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--tune", action="store_true", help="enable the launch autotuner")
    ap.add_argument("--tune-save", default=None, help="write the tuned launch table here")
    ap.add_argument("--delta", type=float, default=None,
                    help="reliable-update threshold: an update when |r| falls below delta x its maximum since the "
                         "last (default by inner precision: 3e-4 for f32, 0.3 for bf16, 0.1 for f16 and i16)")
    ap.add_argument("--check-every", type=int, default=0,
                    help="CG iterations between host polls of the solver state (0: the library's size rule)")
    ap.add_argument("--fh", action="store_true", help="Feynman-Hellmann propagator pairs instead of single solves")
    ap.add_argument("--physical", action="store_true",
                    help="--fh: physical 4D propagators (sources (1 - c5 D_W) inject(xi), opposite walls)")
    ap.add_argument("--split", action="store_true",
                    help="one rank's share of the workload split 2x2x2 in (y, z, t): face packing, interior and "
                         "exterior hop against the plain hop of the same block")
    ap.add_argument("--sample", type=int, default=13,
                    help="time the launches of one CG iteration in this many (prime to the poll period)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the solves without per-launch HIP events (no roofline figures)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the solver runs each "
              f"propagator on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        # the library's copy kernel on 2 GiB each way: HBM counters of its
        # dispatches calibrate those of the stencil
        from paper_1810_01609_amd import mdwf as M

        n = 1 << 27  # 2 GiB of complex128
        src = torch.ones(n, dtype=torch.complex128, device="cuda")
        dst = torch.empty_like(src)
        ctx = M.Context(0)
        gbs = ctx.copy_bandwidth(src, dst, reps=4)
        ctx.close()
        print(json.dumps({"copy_bytes_each_way": n * 16, "launches": 5, "GB_per_s": gbs}))
        return

    if args.workload == "c5":
        serve_bench(args)
        return
    if args.fh:
        fh_bench(args)
        return
    if args.split:
        split_bench(args)
        return
    if args.dslash_only:
        dslash_bench(args)
        return

    import mdwf_synth as S
    from paper_1810_01609_amd import mdwf as M

    cfg = S.CONFIGS[args.workload]
    if args.inner is None:
        args.inner = "f16" if args.workload in ("c3", "c4") else "f32"
    L, L5 = cfg["L"], cfg["L5"]
    nrhs = 12 if cfg["source"] == "point12" else 1
    act = M.Action.make(L, L5, cfg["b5"], cfg["c5"], cfg["M5"], cfg["mq"])
    t_start = time.perf_counter()
    U = S.gauge_field(L, cfg["eps"], cfg["seed"])
    progress(f"gauge field generated ({time.perf_counter() - t_start:.1f} s)")
    ctx = M.Context(0)
    ctx.tune_mode(1 if args.tune else 0)  # tuning happens in the warm-up steps
    # achievable bandwidth in this run: the library's STREAM-style copy of 4 GiB
    a = torch.ones(1 << 28, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    copy_gbs = ctx.copy_bandwidth(a, b, reps=10)
    del a, b
    torch.cuda.empty_cache()
    progress(f"copy kernel {copy_gbs:.0f} GB/s")
    g = ctx.gauge_load(L, U, precs=("f64", args.inner))
    del U
    eta = torch.zeros((nrhs,) + act.spinor_shape(), dtype=torch.complex128, device="cuda")
    psi = torch.zeros_like(eta)
    opts = M.CGOpts.make(tol=1e-10, inner=args.inner, delta=args.delta, check_every=args.check_every)
    opts64 = M.CGOpts.make(tol=1e-10, inner="f64")

    def sources(n):
        for r in range(n):
            if cfg["source"] == "z2":
                ctx.source_z2(act, cfg["z2_seed"], r, eta[r])
            elif cfg["source"] == "point":
                ctx.source_point(act, (0, 0, 0, 0), 0, 0, eta[r])
            else:  # the 12 spin-colour point sources
                ctx.source_point(act, (0, 0, 0, 0), r // 3, r % 3, eta[r])

    def step(o, n=nrhs):
        sources(n)
        if args.sequential:  # the same RHS solved one after another
            st = []
            for r in range(n):
                st.extend(ctx.solve(g, act, o, eta[r:r + 1], psi[r:r + 1], nrhs=1))
            return st
        return ctx.solve(g, act, o, eta[:n], psi[:n], nrhs=n)

    # plain FP64 CG, one RHS at a time, on the first source (reference rate and
    # iteration count)
    st64, t64 = {"iters": 0, "rel_res_full": None}, float("nan")
    if not args.skip_f64:
        if nrhs == 1:
            step(opts64, 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st64 = step(opts64, 1)[0]
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t
        progress(f"plain FP64 single-RHS solve: {t64:.2f} s, {st64['iters']} iterations")

    for w in range(args.warmup):
        t = time.perf_counter()
        step(opts)
        torch.cuda.synchronize()
        progress(f"warm-up step {w + 1}/{args.warmup}: {time.perf_counter() - t:.2f} s")
    torch.cuda.synchronize()
    # kernel timing: every launch outside the CG loop and every launch of one
    # CG iteration in 13 (start/stop events inside the dispatches; 13 is prime
    # to the host's poll period of 8 iterations, so the samples visit every
    # position between two polls).  Timing costs the c2 solve rate 2.7 % at
    # one iteration in 7, 1.7 % at one in 13; the mean launch time is the same.
    ctx.profile_enable(not args.no_kernel_timing, sample=args.sample)
    ctx.profile_reset()
    lat = []
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        stats.extend(step(opts))
        lat.append(time.perf_counter() - ts)
        progress(f"step {k + 1}/{args.steps}: {lat[-1]:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {k: ctx.profile_read(c) for k, c in
            (("dslash", M.PROF_DSLASH_INNER), ("dslash_f64", M.PROF_DSLASH_F64), ("blas", M.PROF_BLAS),
             ("scalar", M.PROF_SCALAR), ("other", M.PROF_OTHER))}
    ctx.profile_enable(False)
    ok = all(s["converged"] == 1 and s["rel_res_normal"] <= 1e-10 for s in stats)

    d = prof["dslash"]
    avg_ms = d["ms"] / max(d["launches"], 1)
    bytes_per_launch = d["bytes"] / max(d["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    traffic, traffic_note = measured_traffic(args.workload)

    line = {
        "metric": "MDWF CG solves/s at rel-res 1e-10; Dslash HBM GB/s; p50/p99 solve latency",
        "value": args.steps * nrhs / elapsed if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.inner == "f64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {L[0]}x{L[1]}x{L[2]}x{L[3]} L5={L5} Moebius b5={cfg['b5']} "
                         f"c5={cfg['c5']} M5={cfg['M5']} mq={cfg['mq']}, links exp(i{cfg['eps']}H) "
                         f"seed {cfg['seed']}, {cfg['source']} source, even-odd CGNR to 1e-10, "
                         f"{args.inner} inner + f64 reliable updates"),
            "lattice": list(L), "L5": L5, "nrhs": nrhs, "inner": args.inner, "tol": 1e-10, "delta": opts.delta,
            "storage": args.inner, "arithmetic": "f64" if args.inner == "f64" else "f32",
            "fused": not args.sequential,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic,
            "kernel": "dslash5_kernel (fused hop + 5th-dim, inner precision)",
            "avg_launch_ms": avg_ms,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "launches": d["launches"],
            "traffic_note": traffic_note,
            "cache_resident": bool(cfg["L"][0] * cfg["L"][1] * cfg["L"][2] * cfg["L"][3] * L5 * 48 < 256e6),
            "copy_GBs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs if achieved and copy_gbs else None,
            "copy_note": "the library's STREAM-style copy kernel (mdwf_copy_bandwidth), 4 GiB, measured in this run",
        },
        "tflops": (stats_flops(stats, nrhs) / elapsed / 1e12) if ok else None,
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99))},
        "solve": {
            "iters": max(s["iters"] for s in stats[-nrhs:]),
            "reliable_updates": max(s["reliable_updates"] for s in stats[-nrhs:]),
            "rel_res_normal": max(s["rel_res_normal"] for s in stats[-nrhs:]),
            "rel_res_full": max(s["rel_res_full"] for s in stats[-nrhs:]),
            "converged_all": ok,
        },
        "f64_plain_cg": {"solves_per_s": 1.0 / t64 if t64 == t64 else None, "iters": st64["iters"],
                         "rel_res_full": st64["rel_res_full"]},
        "kernel_time_ms_per_step": {k: v["ms"] / args.steps for k, v in prof.items()},
    }
    if args.tune:
        line["config"]["tuned"] = True
        line["tune_entries"] = ctx.tune_entries()
        if args.tune_save:
            ctx.tune_save(args.tune_save)
    if not args.no_cpu_baseline and not args.skip_f64:
        progress("timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(cfg, st64["iters"])
    g.free()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
