"""Benchmark: time to a 1e-8 relative residual on the 1024 x 1024 heteroscedastic workload
(k = 3 components, f = 9 maps), float64 PCG vs mixed precision, plus operator-apply bandwidth.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

One step = one complete mixed-precision solve through the C ABI: operator set-up (stencil
coefficients, per-pixel mixing, the preconditioner's set-up), right-hand side B^T C Y, initial
residual, float32 inner PCG runs inside float64 refinement until ||b - G x|| <= 1e-8 ||b||, and
the statistics.  Inputs (kappa, tau, A, W, Y) are resident in HBM before timing starts.  Both
preconditioners are timed (block-Jacobi, and the Fourier preconditioner with pixel-mean weights),
each for the mixed and the float64 solver; the headline value is the faster mixed solve and
fp64_ms the float64 solve with the same preconditioner.  The roofline object reports the
stand-alone operator apply (float32, the precision of the inner runs), timed with HIP events on
the stream it runs on.  Prints one JSON line.

--mode pmc runs only a device copy of known size, the applies, one solve of each precision with
each preconditioner and stand-alone Fourier preconditioner applications, for hardware-counter runs (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE) that calibrate the
HBM-traffic figure.  --mode sylv runs only the Lanczos-Sylvester workload (1024^2, k = 4, f = 9,
separable noise, common kappa) against PCG on the same system.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import resource
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 rel. residual @1024² k=3 (FP64 vs mixed); operator-apply HBM GB/s"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_apply_f32_het_1024.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2204_08057_amd", "csrc", "sylv_kernels.hip")
FOURIER_SRC = os.path.join(ROOT, "paper_2204_08057_amd", "csrc", "sylv_fourier_impl.h")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash(path: str = KERNEL_SRC) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def apply_bytes_per_pixel(k: int, elem: int, f: int = None) -> int:
    """Algorithmic bytes of one operator apply per pixel: read the k input maps and the per-pixel
    weights once (the k(k+1)/2 packed mixing-block planes, or the f weight maps where those are
    fewer), write the k output maps (stencil halos are reuse, not extra traffic)."""
    wt = k * (k + 1) // 2 if f is None else min(f, k * (k + 1) // 2)
    return (2 * k + wt) * elem


def timed_applies(sy, torch, dp, X, ws, reps):
    """Average duration of one apply launch (ms)."""
    Y = torch.empty_like(X)
    return timed_launches(torch, sy.apply_launcher(dp, X, Y, ws), reps)


def timed_launches(torch, launch, reps):
    """Average duration of one call of `launch` (ms): HIP events around `reps` back-to-back calls
    on the stream they run on.  The launches go through a pre-marshalled callable so that the
    host issues them faster than the GPU runs them (else the events time the Python call)."""
    stream = torch.cuda.current_stream()
    for _ in range(5):
        launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        launch()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps   # ms per launch


def traffic_from_counters(kernel_hash: str):
    """HBM bytes per launch of the float32 apply from the committed counter summary, if it was
    taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        d = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if d.get("kernel_source_sha") != kernel_hash:
        return None
    return d.get("traffic_bytes_per_launch")


def fourier_passes_from_counters():
    """Per-pass duration and DRAM bytes of the Fourier preconditioner's kernels (float32 and
    float64, 1024^2, k = 3) from the committed counter summary, if it was taken on the current
    FFT source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        d = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if d.get("fourier_source_sha") != kernel_source_hash(FOURIER_SRC):
        return None
    out = {}
    for name, v in d.get("fourier_kernels", {}).items():
        gbs = v["algorithmic"] / v["median_us"] / 1e3
        out[name] = {"us": v["median_us"], "algorithmic_bytes": v["algorithmic"],
                     "achieved": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4),
                     "traffic": v["fetch"] + v["write"]}
    return out


def cg_iteration_seconds(sy, torch, dp, Y, ws, precision, precond, n1=40, n2=140, reps=5):
    """Wall time of one conjugate-gradient iteration (fused apply + update + the amortised
    completion checks), measured as the difference between solves stopped after n1 and n2
    iterations divided by n2 - n1, so that set-up and the final residual cancel.  Mixed
    precision: one float32 inner run (refine_max 1, inner tolerance below reach)."""
    def median_time(n):
        o = sy.SolveOptions(tol=1e-15, precision=precision, max_iter=n, refine_max=1,
                            inner_tol=1e-30, precond=precond)
        sy.pcg_solve(dp, Y=Y, opts=o, ws=ws, return_stats=False)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            sy.pcg_solve(dp, Y=Y, opts=o, ws=ws, return_stats=False)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)
    return (median_time(n2) - median_time(n1)) / (n2 - n1)


def cg_iteration_bytes_per_pixel(k: int, elem: int, fourier: bool = False,
                                  nx: int = 1024, scale_planes: int = 0) -> float:
    """Algorithmic bytes of one CG iteration per pixel: the fused apply reads p_old, z and the
    k(k+1)/2 mixing planes and writes p, q, and it advances x (float32: read and write x every
    iteration; float64: every second iteration, reading x and p_(i-2) and writing x, i.e. 1.5 k
    planes per iteration on average).  Block-Jacobi: the update reads r, q and the bfloat16
    factor planes and writes r, z.  Fourier: the update reads r, q and writes r; the three FFT
    passes read r and write the half spectrum, read and write it again (column pass), and read it
    and write z: 6 k planes, the half spectrum being (nx/2 + 1) / (nx/2) planes.  The scaled
    variants' two row passes also read the scale planes (diagonal: k, block: k(k+1)/2)."""
    mk = k * (k + 1) // 2
    x_planes = 2.0 * k if elem == 4 else 1.5 * k
    apply = (4 * k + mk + x_planes) * elem
    if not fourier:
        return apply + 4 * k * elem + mk * 2
    half = (nx // 2 + 1) / (nx // 2)
    return apply + 3 * k * elem + (2 * k + 4 * k * half) * elem + 2 * scale_planes * elem


def cpu_baseline(prob, tol, precond="block"):
    """The oracle (plain float64 CPU PCG with the same preconditioner and stopping rule,
    including assembly of the operator) on the full workload, timed on this host."""
    from oracle import operator as op
    from oracle import pcg as opcg
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    G = op.posterior_precision(prob)
    b = op.rhs(prob)
    res = opcg.pcg(prob, b=b, G=G, tol=tol, max_iter=2000, precond=precond)
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    cores = max(1, int(round(cpu / wall)))
    return dict(value=round(wall * 1e3, 1), unit="ms", cores=cores, kind="oracle",
                sample=f"complete oracle solve of the 1024x1024 workload to {tol:g} "
                       f"(assembly + {precond} PCG, {res['iters']} iterations, "
                       f"relres {res['relres_true']:.2e}); host reports {os.cpu_count()} CPUs")


def oracle_errors(prob, xs, tol=1e-13):
    """Error of each GPU solution against the oracle: its float64 block-Jacobi PCG on the CPU to
    a relative residual of `tol` (error below cond(G) * tol, about 1e-10 here); not timed."""
    import numpy as np
    from oracle import pcg as opcg
    ref = opcg.pcg(prob, tol=tol, max_iter=5000, precond="block")
    x = np.asarray(ref["x"]).reshape(-1)
    nrm = np.linalg.norm(x)
    out = {lb: float(np.linalg.norm(X.detach().cpu().numpy().reshape(-1) - x) / nrm)
           for lb, X in xs.items()}
    out.update(reference=f"oracle float64 block-Jacobi PCG on the CPU to relres {tol:g}",
               oracle_iters=int(ref["iters"]), oracle_relres=float(ref["relres_true"]))
    return out


def oracle_sample(prob, nit=10):
    """Seconds for the oracle's assembly of G and per PCG iteration (block-Jacobi) on `prob`:
    a bounded sample that estimates scale linearly in pixels (sparse operators)."""
    from oracle import operator as op
    from oracle import pcg as opcg
    t0 = time.perf_counter()
    G = op.posterior_precision(prob)
    t1 = time.perf_counter()
    opcg.pcg(prob, G=G, tol=0.0, max_iter=nit, precond="block")
    t2 = time.perf_counter()
    return t1 - t0, (t2 - t1) / nit


def time_solves(sy, torch, probs, Y, B, opts, nrhs, steps, warmup):
    """Median time of `steps` solves after `warmup`, with the last stats."""
    plist = probs if isinstance(probs, list) else [probs]
    ws = torch.empty(sy.workspace_bytes(plist, nrhs, opts), dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        sy.pcg_solve(probs, Y=Y, Bextra=B, opts=opts, nrhs=nrhs, ws=ws, return_stats=False)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        X, stt = sy.pcg_solve(probs, Y=Y, Bextra=B, opts=opts, nrhs=nrhs, ws=ws,
                              return_stats=False)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    ms = statistics.median(times)
    n = len(plist) * nrhs
    st = sy.binding._stats_list(stt, n)
    return ms, st, X


def graph_solve(sy, torch, probs, Y, B, opts, nrhs, steps, warmup):
    """The same solve under the fixed schedule, captured once into a HIP graph and replayed.

    The caps of the fixed schedule come from the adaptive solve: max_iter per (inner) run starts
    at 1.1 x the iterations per run plus 2 and grows until the capped solve converges (refine_max
    = the refinement steps the adaptive solve took).  Each replay re-zeroes x and solves; the
    median replay time is reported, and the replayed result must equal the eager fixed-schedule
    solve bitwise."""
    import math
    plist = probs if isinstance(probs, list) else [probs]
    n = len(plist) * nrhs
    _, st = sy.pcg_solve(probs, Y=Y, Bextra=B, opts=opts, nrhs=nrhs)
    mixed = opts.precision == sy.SYLV_PREC_MIXED
    outer = max(s["outer"] for s in st)
    per_run = max(s["iters"] for s in st) / (outer if mixed else 1)
    m = int(math.ceil(per_run * 1.1)) + 2
    fixed = None
    for _ in range(8):
        cand = dataclasses.replace(opts, max_iter=m, schedule=sy.SYLV_SCHED_FIXED,
                                   refine_max=outer if mixed else opts.refine_max)
        _, stc = sy.pcg_solve(probs, Y=Y, Bextra=B, opts=cand, nrhs=nrhs)
        if all(s["status"] == 0 for s in stc):
            fixed = cand
            break
        m = int(m * 1.15) + 2
    if fixed is None:
        return {"error": "no converging caps found"}
    total = sum(nrhs * p.k * p.n_pix for p in plist)
    X = torch.zeros(total, dtype=torch.float64, device="cuda")
    stats = torch.zeros(n * sy.binding.STATS_BYTES, dtype=torch.uint8, device="cuda")
    ws = torch.empty(sy.workspace_bytes(plist, nrhs, fixed), dtype=torch.uint8, device="cuda")
    launch = sy.solve_launcher(probs, X, stats, ws, Y=Y, Bextra=B, opts=fixed, nrhs=nrhs)

    def solve():
        X.zero_()
        launch()

    solve()
    torch.cuda.synchronize()
    X_eager = X.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        solve()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        solve()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    st_g = sy.stats_list(stats, n)
    out = summarize(statistics.median(times), st_g)
    out.update({"max_iter": fixed.max_iter, "refine_max": fixed.refine_max if mixed else None,
                "equal_to_eager": bool(torch.equal(X, X_eager))})
    del g
    return out


def summarize(ms, st):
    return {"ms": round(ms, 3),
            "iters_max": max(s["iters"] for s in st),
            "iters_sum": sum(s["iters"] for s in st),
            "outer_max": max(s["outer"] for s in st),
            "relres_true_max": max(s["relres_true"] for s in st),
            "all_ok": all(s["status"] == 0 for s in st)}


def bench_masked(sy, torch, steps, warmup, cpu=False):
    """2048^2, k = 4, f = 9, 10 % masked pixels (beyond the last-level cache): mixed precision vs
    float64 solves with the block-Jacobi, the Fourier and the diagonally scaled Fourier
    preconditioner, and the stand-alone applies."""
    from workloads import workload
    prob = workload("masked_2048")[0]
    dp = sy.DeviceProblem.from_numpy(prob)
    Y = torch.as_tensor(prob.Y, device="cuda")
    res = {}
    for pc, suffix in ((sy.SYLV_PC_BLOCK, ""), (sy.SYLV_PC_FOURIER, "_fourier"),
                       (sy.SYLV_PC_FOURIER_DIAG, "_fourier_diag"),
                       (sy.SYLV_PC_FOURIER_BLOCK, "_fourier_block")):
        for label, prec in (("mixed", sy.SYLV_PREC_MIXED), ("f64", sy.SYLV_PREC_F64)):
            o = sy.SolveOptions(tol=1e-8, precision=prec, precond=pc)
            try:
                ms, st, _ = time_solves(sy, torch, dp, Y, None, o, 1, steps, warmup)
            except sy.binding.SylvError as err:   # a preconditioner that does not take this grid
                res[label + suffix] = {"refused": str(err)}
                log(f"masked_2048 {label + suffix}: refused ({err})")
                continue
            res[label + suffix] = summarize(ms, st)
            log(f"masked_2048 {label + suffix}: {res[label + suffix]}")
    # stand-alone applies at a size far beyond the 256 MB last-level cache: the HBM figure
    ws_app = sy.binding.prepare(dp, sy.SYLV_PC_NONE)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    X64 = torch.randn((prob.k, prob.n_pix), generator=gen, dtype=torch.float64, device="cuda")
    for label, X, e in (("apply_f32", X64.float(), 4), ("apply_f64", X64, 8)):
        t = timed_applies(sy, torch, dp, X, ws_app, 50)
        nb = apply_bytes_per_pixel(prob.k, e, prob.f) * prob.n_pix
        res[label] = {"us": round(t * 1e3, 2), "algorithmic_bytes": nb,
                      "gbs": round(nb / (t * 1e-3) / 1e9, 1)}
        log(f"masked_2048 {label}: {res[label]}")
    if cpu:
        # the oracle on a 512^2 grid of the same recipe, scaled by the pixel count
        from workloads import make_problem
        small = make_problem(512, 512, prob.k, prob.f, seed=1002, noise="hetero", mask_frac=0.1)
        ta, tit = oracle_sample(small)
        scale = prob.n_pix / small.n_pix
        est = scale * (ta + tit * res["f64"]["iters_max"])
        res["cpu_oracle"] = {"kind": "oracle", "estimate_ms": round(est * 1e3, 0),
                             "sample": "assembly and 10 block-Jacobi PCG iterations of the oracle "
                                       "on a 512^2 grid of the same recipe, scaled by the pixel "
                                       "count (16x) and the float64 GPU run's iteration count"}
        log(f"masked_2048 cpu oracle: {res['cpu_oracle']}")
    return res


def bench_batched(sy, torch, steps, warmup, cpu=False):
    """8 uneven grids x 8 perturbation-optimisation right-hand sides (64 posterior samples):
    independent and block CG, mixed precision and float64."""
    from workloads import WORKLOADS, workload
    probs = workload("batched_8grids")
    nrhs = WORKLOADS["batched_8grids"]["nrhs"]
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    Y = torch.cat([torch.as_tensor(p.Y.ravel(), device="cuda") for p in probs])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1003)
    etas = []
    for p, d in zip(probs, dps):
        xi = torch.randn((nrhs, p.k, p.n_pix), generator=gen, dtype=torch.float64, device="cuda")
        zeta = torch.randn((nrhs, p.f, p.n_pix), generator=gen, dtype=torch.float64,
                           device="cuda")
        etas.append(sy.po_perturb(d, xi, zeta).reshape(-1))
    B = torch.cat(etas)
    res = {}
    for label, prec, blk in (("block_mixed", sy.SYLV_PREC_MIXED, 1),
                             ("independent_mixed", sy.SYLV_PREC_MIXED, 0),
                             ("block_f64", sy.SYLV_PREC_F64, 1),
                             ("independent_f64", sy.SYLV_PREC_F64, 0)):
        o = sy.SolveOptions(tol=1e-8, precision=prec, block=blk)
        ms, st, _ = time_solves(sy, torch, dps, Y, B, o, nrhs, steps, warmup)
        res[label] = summarize(ms, st)
        log(f"batched_8grids {label}: {res[label]}")
    # the configuration chosen by the autotuner (whole solves timed per candidate)
    base = sy.SolveOptions(tol=1e-8, precision=sy.SYLV_PREC_MIXED)
    tuned, tres = sy.autotune(dps, Y=Y, Bextra=B, opts=base, nrhs=nrhs)
    ms, st, _ = time_solves(sy, torch, dps, Y, B, tuned, nrhs, steps, warmup)
    res["autotuned_mixed"] = dict(summarize(ms, st), block=tuned.block,
                                  block_size=tuned.block_size, apply_rows=tuned.apply_rows,
                                  candidates=tres["candidates"])
    log(f"batched_8grids autotuned_mixed: {res['autotuned_mixed']}")
    # the block-CG batch and the autotuner's choice, each as one graph launch (fixed schedule)
    o = sy.SolveOptions(tol=1e-8, precision=sy.SYLV_PREC_MIXED, block=1)
    res["graph_block_mixed"] = graph_solve(sy, torch, dps, Y, B, o, nrhs, steps, warmup)
    log(f"batched_8grids graph_block_mixed: {res['graph_block_mixed']}")
    res["graph_autotuned_mixed"] = graph_solve(sy, torch, dps, Y, B, tuned, nrhs, steps, warmup)
    log(f"batched_8grids graph_autotuned_mixed: {res['graph_autotuned_mixed']}")
    res["right_hand_sides"] = len(probs) * nrhs
    res["pixels"] = sum(p.n_pix for p in probs)
    # effective bandwidth of the independent-CG solves: every instance's iterations times the
    # algorithmic bytes of one iteration on its grid (set-up, right-hand sides, residual and
    # refinement passes not counted, so this is a lower bound of the bytes moved)
    for label, elem in (("independent_mixed", 4), ("independent_f64", 8)):
        _, st, _ = time_solves(sy, torch, dps, Y, B, sy.SolveOptions(
            tol=1e-8, precision=sy.SYLV_PREC_MIXED if elem == 4 else sy.SYLV_PREC_F64), nrhs,
            1, 0)
        nb = sum(st[g * nrhs + r]["iters"] * cg_iteration_bytes_per_pixel(p.k, elem) * p.n_pix
                 for g, p in enumerate(probs) for r in range(nrhs))
        res[label]["cg_bytes"] = int(nb)
        res[label]["gbs_effective"] = round(nb / (res[label]["ms"] * 1e-3) / 1e9, 1)
        log(f"batched_8grids {label}: {res[label]['gbs_effective']} GB/s effective")
    if cpu:
        # the oracle on the batch's smallest grid, scaled by pixels, right-hand sides and the
        # float64 independent-CG iteration count (one assembly per grid)
        ta, tit = oracle_sample(probs[0])
        scale = res["pixels"] / probs[0].n_pix
        est = scale * (ta + tit * nrhs * res["independent_f64"]["iters_max"])
        res["cpu_oracle"] = {"kind": "oracle", "estimate_ms": round(est * 1e3, 0),
                             "sample": f"assembly and 10 block-Jacobi PCG iterations of the oracle "
                                       f"on the {probs[0].ny}^2 grid, scaled by the batch's pixel "
                                       f"count, {nrhs} right-hand sides per grid and the float64 "
                                       "GPU run's iteration count"}
        log(f"batched_8grids cpu oracle: {res['cpu_oracle']}")
    return res


def bench_other_workloads(sy, torch, steps, warmup, cpu=False):
    """The other workloads of the solver, timed the same way (not the headline value)."""
    from workloads import WORKLOADS, workload
    out = {"masked_2048": bench_masked(sy, torch, steps, warmup, cpu=cpu),
           "batched_8grids": bench_batched(sy, torch, steps, warmup, cpu=cpu)}
    # 512^2, k = 4, f = 9: forward solve + adjoint (gradients w.r.t. kappa, tau, A, W, Y)
    prob = workload("grad_512")[0]
    dp = sy.DeviceProblem.from_numpy(prob)
    Y = torch.as_tensor(prob.Y, device="cuda")
    o = sy.SolveOptions(tol=WORKLOADS["grad_512"]["tol"], precision=sy.SYLV_PREC_F64)
    ms_f, st, X = time_solves(sy, torch, dp, Y, None, o, 1, steps, warmup)
    gbar = torch.randn_like(X)
    ws = torch.empty(sy.workspace_bytes([dp], 1, o), dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        sy.pcg_backward(dp, Y, X, gbar, o, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, g, stb = sy.pcg_backward(dp, Y, X, gbar, o, ws=ws)
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) / steps * 1e3
    out["grad_512"] = {"forward": summarize(ms_f, st), "backward_ms": round(ms_b, 3),
                       "backward_iters": stb["iters"], "backward_ok": stb["status"] == 0}
    for key, pcf in (("fourier", sy.SYLV_PC_FOURIER), ("fourier_diag", sy.SYLV_PC_FOURIER_DIAG),
                     ("fourier_block", sy.SYLV_PC_FOURIER_BLOCK)):
        of = dataclasses.replace(o, precond=pcf)
        ms_ff, stf, Xf = time_solves(sy, torch, dp, Y, None, of, 1, steps, warmup)
        wsf = torch.empty(sy.workspace_bytes([dp], 1, of), dtype=torch.uint8, device="cuda")
        for _ in range(warmup):
            sy.pcg_backward(dp, Y, Xf, gbar, of, ws=wsf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, gf, stbf = sy.pcg_backward(dp, Y, Xf, gbar, of, ws=wsf)
        torch.cuda.synchronize()
        out["grad_512"][key] = {
            "forward": summarize(ms_ff, stf),
            "backward_ms": round((time.perf_counter() - t0) / steps * 1e3, 3),
            "backward_iters": stbf["iters"], "backward_ok": stbf["status"] == 0,
            "grad_rel_diff_vs_block": {kk: float(torch.linalg.norm(gf[kk] - g[kk]) /
                                                 max(float(torch.linalg.norm(g[kk])), 1e-300))
                                       for kk in g}}
        del wsf
    log(f"grad_512: {out['grad_512']}")
    if cpu:
        # the oracle at full size: assembly and 10 PCG iterations (scaled to the forward and
        # adjoint iteration counts of the GPU run) plus its gradient contractions, timed once
        from oracle import grad as og
        ta, tit = oracle_sample(prob)
        xg = X.detach().cpu().numpy().reshape(prob.k, prob.n_pix)
        lg = torch.randn_like(X).cpu().numpy().reshape(prob.k, prob.n_pix)
        t0 = time.perf_counter()
        og.implicit_grads(prob, xg, lg)
        tg = time.perf_counter() - t0
        est = ta + tit * (st[0]["iters"] + stb["iters"]) + tg
        out["grad_512"]["cpu_oracle"] = {
            "kind": "oracle", "estimate_ms": round(est * 1e3, 0),
            "gradient_contractions_ms": round(tg * 1e3, 1),
            "sample": "assembly and 10 block-Jacobi PCG iterations of the oracle at 512^2, scaled "
                      "to the GPU run's forward + adjoint iteration counts, plus the oracle's "
                      "gradient contractions at full size"}
        log(f"grad_512 cpu oracle: {out['grad_512']['cpu_oracle']}")
    out["sylv_1024"] = bench_sylvester(sy, torch, steps, warmup, cpu=cpu)
    out["healpix_sky_1024"] = bench_sky(sy, torch, steps, warmup, cpu=cpu)
    out["sweep_1024"] = bench_sweep(sy, torch)
    return out


def bench_sweep(sy, torch):
    """Ten solves over a hyperparameter sweep (kappa +1 %, tau -1 % per step) at 1024^2, k = 3,
    f = 9, to 1e-8 relative to ||b||: each solve from zero, or warm-started from the previous
    solution, with either preconditioner.  Total time and iterations of the sweep."""
    from workloads import WORKLOADS, sweep_parameters, workload
    cfg = WORKLOADS["sweep_1024"]
    prob = workload("sweep_1024")[0]
    params = sweep_parameters(prob, cfg["steps"], cfg["dk"], cfg["dt"])
    Y = torch.as_tensor(prob.Y, device="cuda")
    dp = sy.DeviceProblem.from_numpy(prob)
    res = {"steps": cfg["steps"], "dk": cfg["dk"], "dt": cfg["dt"]}
    for label, prec, pc in (("mixed", sy.SYLV_PREC_MIXED, sy.SYLV_PC_BLOCK),
                            ("f64", sy.SYLV_PREC_F64, sy.SYLV_PC_BLOCK),
                            ("mixed_fourier", sy.SYLV_PREC_MIXED, sy.SYLV_PC_FOURIER),
                            ("f64_fourier", sy.SYLV_PREC_F64, sy.SYLV_PC_FOURIER),
                            ("mixed_fourier_diag", sy.SYLV_PREC_MIXED, sy.SYLV_PC_FOURIER_DIAG),
                            ("f64_fourier_diag", sy.SYLV_PREC_F64, sy.SYLV_PC_FOURIER_DIAG),
                            ("mixed_fourier_block", sy.SYLV_PREC_MIXED, sy.SYLV_PC_FOURIER_BLOCK),
                            ("f64_fourier_block", sy.SYLV_PREC_F64, sy.SYLV_PC_FOURIER_BLOCK)):
        o = sy.SolveOptions(tol=cfg["tol"], precision=prec, stop_ref=sy.SYLV_STOP_B, precond=pc)
        ws = torch.empty(sy.workspace_bytes([dp], 1, o), dtype=torch.uint8, device="cuda")
        for mode in ("cold", "warm"):
            for rep in range(2):            # the first pass warms up
                X = None
                iters, worst = 0, 0.0
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for kap, tau in params:
                    dp.kappa.copy_(torch.as_tensor(kap))
                    dp.tau.copy_(torch.as_tensor(tau))
                    X, st = sy.pcg_solve(dp, Y=Y, X0=X if mode == "warm" else None, opts=o,
                                         ws=ws)
                    iters += st[0]["iters"]
                    worst = max(worst, st[0]["relres_true"])
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
            res[f"{label}_{mode}"] = {"ms": round(ms, 3), "iters_total": iters,
                                      "relres_true_max": worst}
            log(f"sweep_1024 {label} {mode}: {res[f'{label}_{mode}']}")
    return res


def bench_sky(sy, torch, steps, warmup, cpu=False):
    """A full sky at HEALPix level 10: 12 independent 1024^2 faces (links only inside a face),
    k = 4, f = 9, solved in one batched call to 1e-8, mixed precision and float64, with the
    block-Jacobi preconditioner and with the pixel-mean preconditioner in the cosine basis."""
    from workloads import WORKLOADS, workload
    probs = workload("healpix_sky_1024")
    tol = WORKLOADS["healpix_sky_1024"]["tol"]
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    Y = torch.cat([torch.as_tensor(p.Y.ravel(), device="cuda") for p in probs])
    res = {"faces": len(probs), "pixels_per_map": sum(p.n_pix for p in probs)}
    for pc, suffix in ((sy.SYLV_PC_BLOCK, ""), (sy.SYLV_PC_FOURIER, "_cosine"),
                       (sy.SYLV_PC_FOURIER_DIAG, "_cosine_diag"),
                       (sy.SYLV_PC_FOURIER_BLOCK, "_cosine_block")):
        for label, prec in (("mixed", sy.SYLV_PREC_MIXED), ("f64", sy.SYLV_PREC_F64)):
            o = sy.SolveOptions(tol=tol, precision=prec, precond=pc)
            ms, st, _ = time_solves(sy, torch, dps, Y, None, o, 1, steps, warmup)
            res[label + suffix] = summarize(ms, st)
            log(f"healpix_sky_1024 {label + suffix}: {res[label + suffix]}")
    if cpu:
        # the oracle's PCG (assembled sparse G, block-Jacobi) on one full-size face, bounded
        from oracle import operator as op
        from oracle import pcg as opcg
        p0 = probs[0]
        t0 = time.perf_counter()
        G = op.posterior_precision(p0)
        t1 = time.perf_counter()
        nit = 20
        opcg.pcg(p0, G=G, tol=0.0, max_iter=nit, precond="block")
        t2 = time.perf_counter()
        per_it = (t2 - t1) / nit
        est = 12 * ((t1 - t0) + per_it * res["f64"]["iters_max"])
        res["cpu_oracle"] = {"kind": "oracle", "assembly_ms_per_face": round((t1 - t0) * 1e3, 1),
                             "ms_per_iteration_per_face": round(per_it * 1e3, 1),
                             "estimate_full_sky_ms": round(est * 1e3, 0),
                             "sample": f"assembly and {nit} PCG iterations of the oracle on one "
                                       "1024^2 face; the estimate scales them to 12 faces and "
                                       "the float64 GPU run's iteration count"}
        log(f"healpix_sky_1024 cpu oracle: {res['cpu_oracle']}")
    return res


def bench_sylvester(sy, torch, steps, warmup, max_iter=800, cpu=False):
    """1024^2, k = 4, f = 9, separable noise, common kappa: the Lanczos-Sylvester solver
    (Alg. 4 + Alg. 5) against float64 and mixed PCG on the same system, all to 1e-8."""
    from workloads import WORKLOADS, workload
    prob = workload("sylv_1024")[0]
    tol = WORKLOADS["sylv_1024"]["tol"]
    t, n = prob.meta["t"], prob.meta["n"]
    sp = sy.SepProblem.from_numpy(prob.ny, prob.nx, prob.kappa[0], prob.tau, prob.A, t, n)
    Y = torch.as_tensor(prob.Y, device="cuda")
    X = torch.empty((prob.k, prob.n_pix), dtype=torch.float64, device="cuda")
    res = {}
    # the basis kept in HBM (one streaming assembly pass) and Alg. 5's second Lanczos pass (two
    # kept blocks; the recurrence runs again from the kept coefficients)
    for label, mode in (("lanczos_sylvester", sy.SYLV_LZ_KEEP_BASIS),
                        ("lanczos_sylvester_rerun", sy.SYLV_LZ_RERUN)):
        lo = sy.LanczosOptions(tol=tol, max_iter=max_iter, assembly=mode)
        ws = torch.empty(sy.lanczos_workspace_bytes(sp, lo), dtype=torch.uint8, device="cuda")
        Xm = X if mode == sy.SYLV_LZ_KEEP_BASIS else torch.empty_like(X)
        for _ in range(warmup):
            sy.lanczos_solve(sp, Y, lo, ws=ws, out=Xm)
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            t0 = time.perf_counter()
            _, st = sy.lanczos_solve(sp, Y, lo, ws=ws, out=Xm)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        res[label] = {"ms": round(statistics.median(times), 3), "iters": st["iters"],
                      "relres_est": st["relres_est"], "relres_true": st["relres_true"],
                      "ok": st["status"] == 0, "assembly": st["assembly"],
                      "workspace_gb": round(ws.numel() / 1e9, 3)}
        if mode == sy.SYLV_LZ_RERUN:
            res[label]["equal_to_kept_basis"] = bool(torch.equal(Xm, X))
        log(f"sylv_1024 {label}: {res[label]}")
        del ws
    dp = sy.DeviceProblem.from_numpy(prob)
    xs = {"lanczos_sylvester": X}
    for label, prec, pc in (("pcg_f64", sy.SYLV_PREC_F64, sy.SYLV_PC_BLOCK),
                            ("pcg_mixed", sy.SYLV_PREC_MIXED, sy.SYLV_PC_BLOCK),
                            ("pcg_fourier_f64", sy.SYLV_PREC_F64, sy.SYLV_PC_FOURIER),
                            ("pcg_fourier_mixed", sy.SYLV_PREC_MIXED, sy.SYLV_PC_FOURIER),
                            ("pcg_fourier_diag_f64", sy.SYLV_PREC_F64, sy.SYLV_PC_FOURIER_DIAG),
                            ("pcg_fourier_diag_mixed", sy.SYLV_PREC_MIXED,
                             sy.SYLV_PC_FOURIER_DIAG),
                            ("pcg_fourier_block_f64", sy.SYLV_PREC_F64, sy.SYLV_PC_FOURIER_BLOCK),
                            ("pcg_fourier_block_mixed", sy.SYLV_PREC_MIXED,
                             sy.SYLV_PC_FOURIER_BLOCK)):
        o = sy.SolveOptions(tol=tol, precision=prec, precond=pc)
        ms, stl, Xc = time_solves(sy, torch, dp, Y, None, o, 1, steps, warmup)
        res[label] = summarize(ms, stl)
        xs[label] = Xc.reshape(prob.k, prob.n_pix)
        log(f"sylv_1024 {label}: {res[label]}")
    xref = xs["pcg_f64"]
    res["rel_diff_lanczos_vs_pcg_f64"] = float(torch.linalg.norm(X - xref) /
                                               torch.linalg.norm(xref))
    # the paper's comparison method (Alg. 3) with conjugate-gradient column solves on the GPU:
    # the column tolerance is the largest of tol / 2^i whose result meets tol on eq. (Axb)
    # (searched untimed), then the solve is timed like the others
    for label, dec, prec in (("kohler_schur_f64", 0, sy.SYLV_PREC_F64),
                             ("kohler_decoupled_f64", 1, sy.SYLV_PREC_F64),
                             ("kohler_schur_mixed", 0, sy.SYLV_PREC_MIXED),
                             ("kohler_decoupled_mixed", 1, sy.SYLV_PREC_MIXED)):
        ctol = tol
        for _ in range(6):
            o = sy.SolveOptions(tol=ctol, precision=prec)
            _, stk, rr = sy.kohler_solve(sp, Y, o, decouple=bool(dec))
            if rr <= tol:
                break
            ctol /= 2
        kws = torch.empty(sy.kohler_workspace_bytes(sp, bool(dec), o), dtype=torch.uint8,
                          device="cuda")
        for _ in range(warmup):
            sy.kohler_solve(sp, Y, o, decouple=bool(dec), ws=kws)
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            t0 = time.perf_counter()
            Xk, stk, rr = sy.kohler_solve(sp, Y, o, decouple=bool(dec), ws=kws)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        res[label] = {"ms": round(statistics.median(times), 3), "column_tol": ctol,
                      "relres_true": rr, "column_iters": [c["iters"] for c in stk],
                      "ok": all(c["status"] == 0 for c in stk) and rr <= tol,
                      "rel_diff_vs_pcg_f64": float(torch.linalg.norm(Xk - xref) /
                                                   torch.linalg.norm(xref)),
                      "workspace_gb": round(kws.numel() / 1e9, 3)}
        log(f"sylv_1024 {label}: {res[label]}")
        del kws
    res["kappa"] = float(prob.kappa[0])
    if cpu:
        # the oracle's Alg. 5 (eigendecomposition of T_i every step, second Lanczos pass) on
        # the same full-size problem, for a bounded number of steps
        from oracle import lanczos as olz
        nsteps = 25
        t0 = time.perf_counter()
        olz.lanczos_sylvester(prob, t, n, tol=1e-300, max_iter=nsteps)
        wall = time.perf_counter() - t0
        res["cpu_oracle"] = {"kind": "oracle", "ms": round(wall * 1e3, 1), "steps": nsteps,
                             "ms_per_step": round(wall * 1e3 / nsteps, 2),
                             "sample": f"first {nsteps} of {st['iters']} steps of the oracle's "
                                       "Alg. 5 at full size, with its assembly pass"}
        log(f"sylv_1024 cpu oracle: {res['cpu_oracle']}")
    return res


def pmc_workload(sy, torch, mode):
    """Short runs for hardware-counter passes (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE), each
    with a 256 MiB device copy that calibrates the counters.
    pmc_block: 20 iterations of block CG (all 8 columns of every group active throughout) and of
    independent CG on the 8-grid batch, mixed and float64.  pmc_masked: 3 stand-alone applies of
    each precision and one mixed and one float64 solve of the 2048^2 masked workload."""
    from workloads import WORKLOADS, workload
    nbytes = 256 << 20
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    out = {"mode": mode, "copy_bytes": nbytes}
    if mode == "pmc_block":
        probs = workload("batched_8grids")
        nrhs = WORKLOADS["batched_8grids"]["nrhs"]
        dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
        Y = torch.cat([torch.as_tensor(p.Y.ravel(), device="cuda") for p in probs])
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1003)
        B = torch.cat([torch.randn((nrhs, p.k, p.n_pix), generator=gen, dtype=torch.float64,
                                   device="cuda").reshape(-1) for p in probs])
        for prec in (sy.SYLV_PREC_MIXED, sy.SYLV_PREC_F64):
            for blk in (1, 0):
                o = sy.SolveOptions(tol=1e-14, max_iter=20, precision=prec, block=blk,
                                    refine_max=1, inner_tol=1e-30)
                sy.pcg_solve(dps, Y=Y, Bextra=B, opts=o, nrhs=nrhs)
        torch.cuda.synchronize()
        out["pixels"] = sum(p.n_pix for p in probs)
        out["k"], out["s"] = probs[0].k, nrhs
    else:
        prob = workload("masked_2048")[0]
        dp = sy.DeviceProblem.from_numpy(prob)
        Y = torch.as_tensor(prob.Y, device="cuda")
        ws_app = sy.binding.prepare(dp, sy.SYLV_PC_NONE)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(7)
        X64 = torch.randn((prob.k, prob.n_pix), generator=gen, dtype=torch.float64, device="cuda")
        X32 = X64.float()
        for _ in range(3):
            sy.apply(dp, X32, ws=ws_app, prepared=True)
            sy.apply(dp, X64, ws=ws_app, prepared=True)
        for prec in (sy.SYLV_PREC_MIXED, sy.SYLV_PREC_F64):
            sy.pcg_solve(dp, Y=Y, opts=sy.SolveOptions(tol=1e-8, precision=prec))
        torch.cuda.synchronize()
        out["apply_f32_bytes"] = apply_bytes_per_pixel(prob.k, 4, prob.f) * prob.n_pix
        out["apply_f64_bytes"] = apply_bytes_per_pixel(prob.k, 8, prob.f) * prob.n_pix
    out["kernel_source_sha"] = kernel_source_hash()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--apply-reps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 2048^2, batched and differentiable workloads")
    ap.add_argument("--mode", default="bench",
                    choices=["bench", "pmc", "pmc_block", "pmc_masked", "sylv", "sky", "sweep",
                             "masked", "batched"],
                    help="pmc: copy + applies + solves + Fourier applications (counter runs); "
                         "sylv: only the Lanczos-Sylvester workload; sky: only the 12-face "
                         "full-sky workload; sweep: only the hyperparameter sweep; masked: only "
                         "the 2048^2 masked workload; batched: only the 8-grid batch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2204_08057_amd as sy
    from workloads import WORKLOADS, workload

    torch.cuda.set_device(0)
    if args.mode in ("pmc_block", "pmc_masked"):
        print(json.dumps(pmc_workload(sy, torch, args.mode)), flush=True)
        return
    if args.mode == "sylv":
        print(json.dumps({"mode": "sylv", "sylv_1024": bench_sylvester(
            sy, torch, max(2, args.steps // 2), max(1, args.warmup))}), flush=True)
        return
    if args.mode == "batched":
        print(json.dumps({"mode": "batched", "batched_8grids": bench_batched(
            sy, torch, args.steps, args.warmup)}), flush=True)
        return
    if args.mode == "masked":
        print(json.dumps({"mode": "masked", "masked_2048": bench_masked(
            sy, torch, args.steps, args.warmup)}), flush=True)
        return
    if args.mode == "sweep":
        print(json.dumps({"mode": "sweep", "sweep_1024": bench_sweep(sy, torch)}), flush=True)
        return
    if args.mode == "sky":
        print(json.dumps({"mode": "sky", "healpix_sky_1024": bench_sky(
            sy, torch, max(2, args.steps // 2), max(1, args.warmup))}), flush=True)
        return
    name = "het_1024"
    cfg = WORKLOADS[name]
    prob = workload(name)[0]
    k, f, n_pix = prob.k, prob.f, prob.n_pix
    dp = sy.DeviceProblem.from_numpy(prob)
    Y = torch.as_tensor(prob.Y, device="cuda")
    tol = cfg["tol"]
    rng = np.random.default_rng(3)
    X64 = torch.as_tensor(rng.standard_normal((k, n_pix)), device="cuda")
    X32 = X64.to(torch.float32)
    ws_app = sy.binding.prepare(dp, sy.SYLV_PC_NONE)

    if args.mode == "pmc":
        nbytes = 256 << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        for _ in range(3):
            sy.apply(dp, X32, ws=ws_app, prepared=True)
            sy.apply(dp, X64, ws=ws_app, prepared=True)
        # one solve of each precision with each preconditioner (block-Jacobi, Fourier, scaled
        # Fourier), so that the counters also cover the CG kernels and the FFT passes, and three
        # stand-alone Fourier applications of each precision
        for pc in (sy.SYLV_PC_BLOCK, sy.SYLV_PC_FOURIER, sy.SYLV_PC_FOURIER_DIAG,
                   sy.SYLV_PC_FOURIER_BLOCK):
            for prec in (sy.SYLV_PREC_MIXED, sy.SYLV_PREC_F64):
                sy.pcg_solve(dp, Y=Y, opts=sy.SolveOptions(tol=tol, precision=prec, precond=pc))
        ws_fp = sy.binding.prepare(dp, sy.SYLV_PC_FOURIER)
        for R in (X32, X64):
            launch = sy.precond_launcher(dp, R, torch.empty_like(R), sy.SYLV_PC_FOURIER, ws_fp)
            for _ in range(3):
                launch()
        torch.cuda.synchronize()
        print(json.dumps({"mode": "pmc", "copy_bytes": nbytes,
                          "apply_f32_bytes": apply_bytes_per_pixel(k, 4, f) * n_pix,
                          "apply_f64_bytes": apply_bytes_per_pixel(k, 8, f) * n_pix,
                          "kernel_source_sha": kernel_source_hash()}))
        return

    # the preconditioners the library offers for this periodic grid; the headline is the
    # fastest mixed-precision solve, and the float64 figure is quoted with the same preconditioner
    preconds = {"block": (sy.SYLV_PC_BLOCK, "block-Jacobi"),
                "fourier": (sy.SYLV_PC_FOURIER, "Fourier (pixel-mean weights, per-mode inverse)"),
                "fourier_diag": (sy.SYLV_PC_FOURIER_DIAG,
                                 "Fourier with diagonal scaling (pixel-mean weights, per-mode "
                                 "inverse, scaled per pixel to the diagonal of G)"),
                "fourier_block": (sy.SYLV_PC_FOURIER_BLOCK,
                                  "Fourier with block scaling (pixel-mean weights, per-mode "
                                  "inverse, transformed per pixel to G's k x k pixel blocks)")}
    opts = {(label, pc): sy.SolveOptions(tol=tol, precision=prec, precond=preconds[pc][0])
            for pc in preconds
            for label, prec in (("mixed", sy.SYLV_PREC_MIXED), ("f64", sy.SYLV_PREC_F64))}
    ws_bytes = max(sy.workspace_bytes([dp], 1, o) for o in opts.values())
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    results = {}
    for key, o in opts.items():
        for _ in range(args.warmup):
            sy.pcg_solve(dp, Y=Y, opts=o, ws=ws, return_stats=False)
        torch.cuda.synchronize()
        times = []
        t_all = time.perf_counter()
        for _ in range(args.steps):
            t0 = time.perf_counter()
            X, stats_t = sy.pcg_solve(dp, Y=Y, opts=o, ws=ws, return_stats=False)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        ms_mean = (time.perf_counter() - t_all) / args.steps * 1e3
        ms = statistics.median(times)
        st = sy.binding._stats_list(stats_t, 1)[0]
        results[key] = dict(ms=ms, ms_mean=ms_mean, stats=st, X=X)
        log(f"{key}: median {ms:.3f} ms/solve (mean {ms_mean:.3f})  {st}")
    best = min(preconds, key=lambda pc: results[("mixed", pc)]["ms"])

    # the same solves captured once into a HIP graph (fixed schedule) and replayed
    graph = {}
    for label, pc in opts:
        graph[f"{label}_{pc}"] = graph_solve(sy, torch, dp, Y, None, opts[(label, pc)], 1,
                                             args.steps, args.warmup)
        log(f"graph replay {label} {pc}: {graph[f'{label}_{pc}']}")

    # secondary check, GPU against GPU: float64 PCG to a 1e-12 relative residual (not timed)
    xref, st_ref = sy.pcg_solve(dp, Y=Y, ws=ws, opts=sy.SolveOptions(
        tol=1e-12, precision=sy.SYLV_PREC_F64, precond=sy.SYLV_PC_BLOCK))
    nref = torch.linalg.norm(xref)
    err_gpu = {f"{lb}_{pc}": float(torch.linalg.norm(results[(lb, pc)]["X"] - xref) / nref)
               for lb, pc in results}
    log(f"error vs GPU float64 tol 1e-12 (relres {st_ref[0]['relres_true']:.2e}): {err_gpu}")

    t32 = timed_applies(sy, torch, dp, X32, ws_app, args.apply_reps)
    t64 = timed_applies(sy, torch, dp, X64, ws_app, args.apply_reps)
    b32 = apply_bytes_per_pixel(k, 4, f) * n_pix
    b64 = apply_bytes_per_pixel(k, 8, f) * n_pix
    gbs32 = b32 / (t32 * 1e-3) / 1e9
    gbs64 = b64 / (t64 * 1e-3) / 1e9
    log(f"apply f32 {t32 * 1e3:.2f} us {gbs32:.0f} GB/s; f64 {t64 * 1e3:.2f} us {gbs64:.0f} GB/s")

    # the stand-alone Fourier preconditioner (three FFT passes with the per-mode solve), float32
    ws_fp = sy.binding.prepare(dp, sy.SYLV_PC_FOURIER)
    Zf = torch.empty_like(X32)
    t_fp = timed_launches(torch, sy.precond_launcher(dp, X32, Zf, sy.SYLV_PC_FOURIER, ws_fp),
                          args.apply_reps)
    b_fp = int(6 * k * 4 * n_pix * (prob.nx // 2 + 1) / (prob.nx // 2))
    log(f"Fourier preconditioner f32 {t_fp * 1e3:.2f} us {b_fp / t_fp / 1e6:.0f} GB/s")
    # the block-scaled one (the headline's): the row passes also read the k(k+1)/2 planes of T
    ws_fb = sy.binding.prepare(dp, sy.SYLV_PC_FOURIER_BLOCK)
    t_fb = timed_launches(torch, sy.precond_launcher(dp, X32, Zf, sy.SYLV_PC_FOURIER_BLOCK,
                                                     ws_fb), args.apply_reps)
    b_fb = b_fp + 2 * (k * (k + 1) // 2) * 4 * n_pix
    log(f"block-scaled Fourier preconditioner f32 {t_fb * 1e3:.2f} us "
        f"{b_fb / t_fb / 1e6:.0f} GB/s")
    del ws_fb

    # the dominant loop: one CG iteration, timed live for both precisions and preconditioners
    cg_it = {}
    for pc in preconds:
        for label, prec, elem in (("f32", sy.SYLV_PREC_MIXED, 4), ("f64", sy.SYLV_PREC_F64, 8)):
            # Fourier runs reach the float32 floor within ~10 iterations: time 3 against 11
            n1, n2 = (40, 140) if pc == "block" else (3, 11)
            sec = cg_iteration_seconds(sy, torch, dp, Y, ws, prec, preconds[pc][0], n1, n2)
            planes = {"fourier_diag": k, "fourier_block": k * (k + 1) // 2}.get(pc, 0)
            nb = int(cg_iteration_bytes_per_pixel(k, elem, pc != "block", prob.nx, planes)
                     * n_pix)
            cg_it[f"{label}_{pc}"] = {
                "us": round(sec * 1e6, 2), "algorithmic_bytes": nb,
                "achieved": round(nb / sec / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(nb / sec / 1e9 / PEAK_HBM_GBS, 4)}
            log(f"CG iteration {label} {pc}: {cg_it[f'{label}_{pc}']}")

    khash = kernel_source_hash()
    traffic = traffic_from_counters(khash)

    head = results[("mixed", best)]
    f64 = results[("f64", best)]
    mixed_ms = head["ms"]
    line = {
        "metric": METRIC,
        "value": round(mixed_ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed_ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 apply + f64 refinement",
        "data": "synthetic",
        "config": {"workload": name, "ny": prob.ny, "nx": prob.nx, "k": k, "f": f,
                   "noise": "heteroscedastic, W = sigma_f^-2 * lognormal(0, 0.5)",
                   "tol": tol, "precond": preconds[best][1], "x0": "zeros"},
        "fp64_ms": round(f64["ms"], 4),
        "speedup_mixed_vs_fp64": round(f64["ms"] / mixed_ms, 3),
        "iters_fp64": f64["stats"]["iters"],
        "iters_mixed_inner": head["stats"]["iters"],
        "outer_mixed": head["stats"]["outer"],
        "relres_true_fp64": f64["stats"]["relres_true"],
        "relres_true_mixed": head["stats"]["relres_true"],
        "by_precond": {pc: {lb: {"ms": round(results[(lb, pc)]["ms"], 4),
                                 "ms_mean": round(results[(lb, pc)]["ms_mean"], 4),
                                 "iters": results[(lb, pc)]["stats"]["iters"],
                                 "outer": results[(lb, pc)]["stats"]["outer"],
                                 "relres_true": results[(lb, pc)]["stats"]["relres_true"]}
                            for lb in ("mixed", "f64")} for pc in preconds},
        "rel_err_vs_ref": None,
        "rel_err_vs_gpu_f64": dict(err_gpu, reference="GPU float64 block-Jacobi PCG to relres "
                                                      "1e-12 (secondary)"),
        "graph_replay": graph,
        "apply_f32_us": round(t32 * 1e3, 3),
        "apply_f64_us": round(t64 * 1e3, 3),
        "apply_f32_gbs": round(gbs32, 1),
        "apply_f64_gbs": round(gbs64, 1),
        "fourier_precond_f32": {"us": round(t_fp * 1e3, 3), "algorithmic_bytes": b_fp,
                                "gbs": round(b_fp / t_fp / 1e6, 1),
                                "note": "one stand-alone call (three FFT passes and the call's "
                                        "two table uploads), HIP events over back-to-back calls"},
        "fourier_block_precond_f32": {"us": round(t_fb * 1e3, 3), "algorithmic_bytes": b_fb,
                                      "gbs": round(b_fb / t_fb / 1e6, 1),
                                      "frac": round(b_fb / t_fb / 1e6 / PEAK_HBM_GBS, 4),
                                      "note": "the headline's preconditioner, one stand-alone "
                                              "call as above; its row passes also read T"},
        "roofline_fourier": {"bound": "hbm", "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "passes": fourier_passes_from_counters(),
                             "source": "median active launch of rocprofv3 --kernel-trace and "
                                       "FETCH_SIZE / WRITE_SIZE runs of bench.py --mode pmc"},
        "roofline": {
            "kernel": "operator apply, float32 (k_apply<float,3,4,plain>)",
            "bound": "hbm",
            "achieved": round(gbs32, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(gbs32 / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": b32,
        },
        "kernel_source_sha": khash,
        "roofline_cg_iteration": dict(cg_it, bound="hbm", note=(
            "fused CG apply + update (+ the three FFT passes with the Fourier preconditioner) + "
            "amortised completion checks per iteration, from solves stopped after 40 and 140 "
            "iterations (block-Jacobi) or 3 and 11 (Fourier); float32 = the inner runs of the "
            "mixed path")),
    }
    if not args.no_extra:
        line["other_workloads"] = bench_other_workloads(sy, torch, max(2, args.steps // 2),
                                                        max(1, args.warmup), cpu=not args.no_cpu)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(prob, tol, best)
        line["rel_err_vs_ref"] = oracle_errors(
            prob, {f"{lb}_{pc}": results[(lb, pc)]["X"] for lb, pc in results})
        log(f"error vs oracle: {line['rel_err_vs_ref']}")
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
