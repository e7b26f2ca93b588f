#!/usr/bin/env python3
"""Benchmark: graph-captured optimisation steps (forward trace + splat, loss, adjoint, Adam) on one GPU.

Prints ONE JSON line.  Default workload: an extended source approximated by a 9 x 9 grid of point sources
over 1 mm x 1 mm, each sampled with 1024 x 1024 strata (84.9 M rays per step), through the plano-freeform
lens with a 32 x 32 bicubic control net onto a 256 x 256 detector (the largest single design; 100 Adam
steps captured in one HIP graph).

  value       forward+adjoint rays per second of whole optimisation steps (inputs resident in HBM)
  roofline    the dominant trace kernel's algorithmic FP32 FLOP/s (per-ray operation counts below) over
              its mean duration, measured with HIP events on the same stream right after the timed region
              (the kernel alone, launched back to back as many times as there are timed steps), against the
              published FP32 vector peak (157.3 TFLOP/s) and, as a secondary figure, the non-packed 78.6
  fd          forward-only central finite-difference gradient over all control points on the same GPU:
              2K perturbed designs traced in one batched launch, and its agreement with the adjoint
  cpu_baseline  the FP64 oracle (forward + loss + forward-mode gradient) on the host cores, on a bounded
              sample of the workload (the same geometry with fewer strata per emitter)
  batch       (default workload only) the 64-design batch of uneven sizes: aggregate rays/s of its
              graph-captured steps, and the same designs as 64 separate plans and graphs

With --generator dense|sparse the optimised variables are the parameters of the control-point generator of
sec. 2.4 (three control-net-sized tanh layers and the output correction onto [Pz - 0.2, Pz + 0.2] mm,
initialised U(-1e-4, 1e-4) as in the paper); each step then also runs the generator's forward pass, its
back-propagation and Adam on its parameters.  The "generator" object gives those kernels' mean durations and
their HBM roofline (algorithmic bytes below); the top-level roofline is that of the longest kernel group.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "forward+adjoint rays/s and Adam steps/s vs finite-diff gradient, same GPU @1e-3"

# Algorithmic FP32 operations per ray (add, mul, compare-free arithmetic; fma = 2; exp, sqrt, rsqrt, rcp,
# sincos = 1 each), counted stage by stage from the kernels' formulation for p = q = 3, nu = 3, with the
# closed-form uniform cubic of interior spans: 27 operations per axis for N and N', 4 more for N''
# (the generic recurrence takes ~42 and ~20).  tests/test_flop_table.py holds the totals against the FP32
# instructions the hardware counted per ray (rocprofv3 SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F32, summaries in
# profiles/); the point-source adjoint's total is that count (its stage-by-stage sum overstated it).
FLOPS = {
    "collimated": {"forward": 320, "adjoint": 525, "newton_iter": 0},
    # point sources: fixed part (with the exit-root bracket) + per Newton iteration (surface value and slope,
    # step).  Inside a step the adjoint of exact-root, flat-entry designs reads the roots the forward stored:
    # it does neither the bracket nor the iterations.
    "point": {"forward": 390, "adjoint": 777, "newton_iter": 194, "bracket": 35},
}
# Plans keep the exit roots for the adjoint when they take at most this many bytes (4 per ray).
ROOTS_CAP_BYTES = 1 << 30
# Triangle mesh (sec. 2.2.2) instead of the root: per visited cell, four span-basis evaluations at the
# cell's nodes (~204), four corner heights (~96) and two plane tests (~30); the adjoint adds the hit cell's
# barycentric basis weights (~64) and re-walks the cells.  A collimated ray visits exactly one cell.
MESH_CELL_FLOPS = 330
MESH_ADJ_EXTRA = 64
# Freeform entry face: the entry root search (bracket, ~2 Newton steps of a surface value and slope), the entry
# normal and refraction; every ray then searches the exit face like a point-source ray.  The adjoint adds the
# entry reverse (second derivatives at the entry hit, the entry refraction, the entry root).
ENTRY_FLOPS = {"forward": 510, "adjoint": 778}
# Algorithmic HBM bytes of the generator per design with K control points and n parameters (fp32): the
# forward reads the two weight matrices (dense 2 K^2, sparse 2 C K floats; vectors of K are negligible); the
# back-propagation reads them again; the gradient + Adam pass reads and writes parameters and both moments
# (6 n floats).
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3            # published FP32 vector peak (packed FMA)
PEAK_FP32_NONPACKED_TFLOPS = 78.6   # 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz without packed FP32


def _sha(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def _traffic(kernel, workload, source="trace.hpp"):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it matches the current source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2302_12031_amd", "csrc", source)
    if fields.get(f"{source} sha256/16") != _sha(src):
        return None
    try:
        return float(fields["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def sample_workload(wl, max_rays=1 << 20):
    """A bounded sample of a workload for the CPU baseline: every design keeps its lens, detector and target,
    with its sample grid (rays per axis, or strata per axis and emitter) shrunk so that the designs together
    trace at most about max_rays rays."""
    from dataclasses import replace

    from paper_2302_12031_amd import workloads as W
    probs = []
    cap = max_rays / len(wl.problems)
    for p in wl.problems:
        per = p.num_rays() // (p.source.grid_u * p.source.grid_v)  # emitters
        side = max(8, min(p.source.grid_u, int((cap / per) ** 0.5) // 8 * 8))
        probs.append(replace(p, source=replace(p.source, grid_u=side, grid_v=side)))
    return W.Workload(wl.name + "-sample", probs, wl.Pz, wl.targets)


def cpu_baseline(wl, budget_s=10.0):
    import oracle
    threads = min(16, len(os.sched_getaffinity(0)))
    sample = sample_workload(wl)
    reps, t0 = 0, time.perf_counter()
    while True:
        for p, Pz, T in zip(sample.problems, sample.Pz, sample.targets):
            oracle.grad(p, Pz, T, threads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 50:
            break
    sides = sorted({p.source.grid_u for p in sample.problems})
    return {"value": sample.num_rays * reps / el, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample.problems)} design(s) of the workload with the same lens, detector and target "
                      f"and {sides} samples (strata per emitter) per axis: {sample.num_rays} rays, forward + loss "
                      f"+ forward-mode gradient in FP64, {reps} repetition(s) in {el:.1f} s"}


def make_workload(args):
    from paper_2302_12031_amd import workloads as W
    if args.workload == "tophat":
        wl = W.tophat()
    elif args.workload == "tophat64":
        wl = W.tophat(rays_side=1024, cps_side=64, det_side=128)
    elif args.rays_side:
        if args.workload not in ("c2", "c3", "c4"):
            sys.exit("--rays-side applies to c2, c3 and c4")
        wl = W.WORKLOADS[args.workload](args.rays_side)
    else:
        wl = W.WORKLOADS[args.workload]()
    if args.mesh:
        wl = W.with_mesh(wl, args.mesh)
    if args.entry_freeform:
        wl = W.with_entry_freeform(wl)
    return wl


def timed_steps(ffrt, wl, steps, warmup, stream, arch=None, shapes=None, autotune=True, autotune_reps=5):
    """Autotune (or set) the kernel shapes, warm up, capture `steps` steps in one graph and time its launch with
    HIP events on `stream`.  Returns the plan, its state, the target and the timings."""
    import torch

    from paper_2302_12031_amd import workloads as W
    plan = ffrt.Plan(wl.problems)
    T = plan.pack_img(wl.targets)
    if arch is None:
        st = plan.new_state(plan.pack_cp(wl.Pz))
    else:
        lo = plan.pack_cp([z - 0.2 for z in wl.Pz])
        span = torch.full_like(lo, 0.4)
        n_par = plan.mlp_offsets(arch)[-1]
        g = torch.Generator().manual_seed(W.STREAM_FD)
        par = ((torch.rand(n_par, generator=g) * 2 - 1) * 1e-4).to(plan.device)
        st = plan.new_mlp_state(par, lo, span, arch=arch)
    if shapes:
        plan.set_config(0, shapes[0])
        plan.set_config(1, shapes[1])
    elif autotune:
        irr = plan.forward(st["Pz"])
        _, dLdI = plan.loss(irr, T)
        plan.autotune(st["Pz"], irr, dLdI, st["dLdP"], reps=autotune_reps)
    capture = ffrt.Plan.graph_capture if arch is None else ffrt.Plan.graph_capture_mlp
    with torch.cuda.stream(stream):
        capture(plan, st, T, steps=1)               # warm-up graph
    torch.cuda.synchronize()
    for _ in range(warmup):
        plan.graph_launch(stream)
    torch.cuda.synchronize()
    timed = ffrt.Plan(wl.problems)
    timed.set_config(0, plan.get_config(0))
    timed.set_config(1, plan.get_config(1))
    with torch.cuda.stream(stream):
        capture(timed, st, T, steps=steps)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    timed.graph_launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    return dict(plan=plan, timed=timed, st=st, T=T, ms_total=ms_total, ms_step=ms_total / steps, t_wall=t_wall,
                cfg=(plan.config_names(0)[plan.get_config(0)], plan.config_names(1)[plan.get_config(1)]))


def mean_search_steps(ffrt, wl, plan, Pz):
    """Mean Newton iterations (or mesh cells) per hit ray of the first design whose rays search the exit face,
    from the per-ray inspection of 4096 rays (the trace kernels do not count them)."""
    import numpy as np

    def searched(p):
        return p.source.kind != 0 or p.lens.entry_freeform

    if not any(searched(p) for p in wl.problems):
        return 0.0
    d0 = next(i for i, p in enumerate(wl.problems) if searched(p))
    ids = np.linspace(0, wl.problems[d0].num_rays() - 1, 4096).astype(np.int64)
    pz0 = Pz[plan.cp_offsets[d0]:plan.cp_offsets[d0 + 1]].contiguous()
    sub = ffrt.Plan([wl.problems[d0]])
    tr = sub.trace_rays(0, pz0, ids).cpu().numpy()
    return float(tr[tr[:, 0] == 0, 7].mean()) if (tr[:, 0] == 0).any() else 0.0


def algorithmic_flops(wl, kernel, iters, steps=None):
    """FP32 operations of one launch of the forward or adjoint trace kernel over the whole workload: a fixed
    part per ray plus a part per search step (Newton iteration, or triangle-mesh cell).  `steps` (per design)
    are the forward's own search-step totals (its statistics); otherwise every searching ray takes `iters`,
    the mean of a per-ray inspection (which starts each search afresh, as the adjoint does)."""
    root_rays = sum(p.num_rays() for p in wl.problems
                    if p.source.kind != 0 and not p.lens.entry_freeform and not p.options.mesh_u)
    roots_reused = 0 < 4 * root_rays <= ROOTS_CAP_BYTES
    tot = 0.0
    for d, p in enumerate(wl.problems):
        k = "collimated" if p.source.kind == 0 and not p.lens.entry_freeform else "point"
        n = p.num_rays()
        if p.lens.entry_freeform:
            f0, fs = FLOPS["point"][kernel] + ENTRY_FLOPS[kernel], FLOPS["point"]["newton_iter"]
        elif p.options.mesh_u:
            f0 = FLOPS[k][kernel] + (MESH_CELL_FLOPS + MESH_ADJ_EXTRA if kernel == "adjoint" else 0)
            fs = MESH_CELL_FLOPS
        elif k == "point" and kernel == "adjoint" and roots_reused:
            f0, fs = FLOPS[k][kernel] - FLOPS[k]["bracket"], 0.0
        else:
            f0, fs = FLOPS[k][kernel], FLOPS[k]["newton_iter"]
        if k == "collimated" and p.options.mesh_u:
            s = float(n)                                # one cell per collimated ray
        elif steps is not None and kernel == "forward":
            s = float(steps[d])
        else:
            s = iters * n
        tot += f0 * n + fs * s
    return tot, roots_reused


def lds_atomic_roofline(ffrt, wl, fstats, fwd_cfg, fwd_ms, stream):
    """The forward's LDS-tile atomics against the chip's measured LDS-atomic throughput (ffrt_lds_atomic_rate:
    distinct banks, and the splat's own access pattern).  Point-source and freeform-entry rays add their
    nu_x x nu_y window per hit; collimated threads add one (nu_x + 1) x (nu_y + 1) window per RPT rays."""
    if "lds-tile" not in fwd_cfg:
        return None
    rpt = int(fwd_cfg.split("rpt")[1].split()[0])
    n = 0.0
    for d, p in enumerate(wl.problems):
        hits = float(fstats["n_hit"][d])
        nu = p.detector.nu_x * p.detector.nu_y
        direct = p.source.kind != 0 or p.lens.entry_freeform or nu > 25
        n += hits * (nu if direct else (p.detector.nu_x + 1) * (p.detector.nu_y + 1) / rpt)
    peak = ffrt.lds_atomic_rate(0, stream=stream)
    splat = ffrt.lds_atomic_rate(1, stream=stream)
    achieved = n / (fwd_ms * 1e-3)
    return {"per_launch": n, "achieved_per_s": achieved, "peak_per_s": peak, "splat_pattern_per_s": splat,
            "frac_of_peak": achieved / peak, "frac_of_splat_pattern": achieved / splat}


def finite_differences(ffrt, W, wl, plan, T, ms_step, with_oracle):
    """Forward-only central differences over every control point of a single-design workload at its initial
    design, on the same GPU, against the adjoint."""
    import numpy as np
    import torch
    p = wl.problems[0]
    K = p.lens.n_u * p.lens.n_v
    P = plan.pack_cp(wl.Pz)
    irr = plan.forward(P)
    _, dLdI = plan.loss(irr, T)
    g_adj = plan.adjoint(P, dLdI).cpu().numpy()
    # h = 1e-4 mm; the losses of the perturbed designs are reduced in double precision (their central
    # difference is ~1e-5 of the loss itself).  A larger step is not an option: at 1e-3 mm the landing
    # points move by ~0.1 pixel and the truncation error of the quotient reaches ~4e-3.
    h = 1e-4
    Pp = P.repeat(K, 1) + h * torch.eye(K, device=P.device)
    Pm = P.repeat(K, 1) - h * torch.eye(K, device=P.device)
    Pfd = torch.stack([Pp, Pm], 1).reshape(-1).contiguous()
    denom = (torch.diagonal(Pp) - torch.diagonal(Pm)).cpu().numpy()   # exact fl(P+h) - fl(P-h)
    del Pp, Pm
    fdplan = ffrt.Plan([p] * (2 * K))
    fdplan.set_config(0, plan.get_config(0))
    Tfd = T.repeat(2 * K)
    irr_fd = torch.empty(fdplan.total_img, device=P.device)
    loss_fd = torch.empty(2 * K, dtype=torch.float64, device=P.device)
    fdplan.forward(Pfd, irr_fd)
    fdplan.loss_f64(irr_fd, Tfd, loss_fd)
    torch.cuda.synchronize()
    reps = 2
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record()
    for _ in range(reps):
        fdplan.forward(Pfd, irr_fd)
        fdplan.loss_f64(irr_fd, Tfd, loss_fd)
    f1.record()
    torch.cuda.synchronize()
    fd_ms = f0.elapsed_time(f1) / reps
    L = loss_fd.cpu().numpy().astype(np.float64)
    g_fd = (L[0::2] - L[1::2]) / denom
    # control points where some ray changes its discrete state (screen edge, TIR, side wall) within +-h:
    # there the difference quotient measures a jump the pathwise derivative leaves out by definition
    st_fd, st0 = fdplan.new_stats(), plan.new_stats()
    fdplan.forward(Pfd, irr_fd, stats=st_fd)
    plan.forward(P, stats=st0)
    S, S0 = fdplan.decode_stats(st_fd), plan.decode_stats(st0)[0]
    keys = ("n_hit", "n_miss_entry", "n_side_wall", "n_tir", "n_off_screen")
    flip = np.array([any(S[2 * k][c] != S0[c] or S[2 * k + 1][c] != S0[c] for c in keys) for k in range(K)])
    clean = np.where(~flip)[0]
    sel = np.random.default_rng(W.STREAM_FD).choice(clean, min(16, len(clean)), replace=False)
    gmax = np.abs(g_adj).max()
    err_clean = float(np.abs(g_fd[clean] - g_adj[clean]).max() / gmax) if len(clean) else float("nan")
    fd = {"h_mm": h, "control_points": K, "rays_per_gradient": 2 * K * wl.num_rays,
          "ms_per_gradient": fd_ms, "speedup_of_step": fd_ms / ms_step,
          "max_rel_err_16cp": float(np.abs(g_fd[sel] - g_adj[sel]).max() / gmax),
          "max_rel_err_all_flip_free": err_clean,
          "max_rel_err_all": float(np.abs(g_fd - g_adj).max() / gmax),
          "agree_at_1e-3": bool(err_clean <= 1e-3),
          "cps_with_state_flips": int(flip.sum()),
          "note": "initial design; FP32 images, losses reduced in FP64; errors relative to max |dL/dP|, over "
                  "control points whose rays keep their discrete state within +-h, and over all"}
    del fdplan, irr_fd, Pfd, Tfd
    if with_oracle:
        import oracle
        _, g64, _, _ = oracle.grad(p, wl.Pz[0], wl.targets[0], threads=min(16, len(os.sched_getaffinity(0))))
        g64 = g64.ravel()
        fd["adjoint_vs_oracle_fp64"] = float(np.abs(g_adj - g64).max() / np.abs(g64).max())
        fd["fd_vs_oracle_fp64_16cp"] = float(np.abs(g_fd[sel] - g64[sel]).max() / np.abs(g64).max())
    return fd


def separate_plans(ffrt, wl, stream, autotune=True):
    """Every design of a batch in a plan and a graph of its own, launched one after another: ms per step."""
    import torch
    sep_ms = 0.0
    k_sep = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for d, p in enumerate(wl.problems):
        pd = ffrt.Plan([p])
        Td = pd.pack_img([wl.targets[d]])
        if autotune:
            P0 = pd.pack_cp([wl.Pz[d]])
            irr0 = pd.forward(P0)
            _, g0 = pd.loss(irr0, Td)
            pd.autotune(P0, irr0, g0, torch.empty_like(P0), reps=3)
        sd = pd.new_state(pd.pack_cp([wl.Pz[d]]))
        with torch.cuda.stream(stream):
            pd.graph_capture(sd, Td, steps=k_sep)
            pd.graph_launch(stream)
        torch.cuda.synchronize()
        e0.record(stream)
        pd.graph_launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        sep_ms += e0.elapsed_time(e1) / k_sep
    return sep_ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4", "c5", "tophat", "tophat64"])
    ap.add_argument("--generator", default="none", choices=["none", "dense", "sparse"])
    ap.add_argument("--rays-side", type=int, default=0,
                    help="rays (collimated) or strata (point sources) per axis, per emitter, instead of the "
                         "workload's own count (c2, c3, c4): the same geometry at another size")
    ap.add_argument("--entry-freeform", action="store_true",
                    help="make the entry face a second freeform B-spline (both nets optimised)")
    ap.add_argument("--mesh", type=int, default=0,
                    help="trace the triangle mesh of sec. 2.2.2 with this many rectangles per knot span and axis")
    ap.add_argument("--no-fd", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="default workload: skip the secondary measurement of the 64-design batch")
    ap.add_argument("--fd-oracle", action="store_true",
                    help="also compare the adjoint and the finite differences with the FP64 oracle's gradient "
                         "(at full size: ~30 s of host time on the C4 workload)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--shapes", default=None,
                    help="forward,adjoint kernel-shape indices to use instead of autotuning (e.g. 0,1)")
    ap.add_argument("--compare-separate", action="store_true",
                    help="multi-design workloads: also time every design in a plan and graph of its own")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB buffer three times (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the tracer runs on a single MI355X "
              "(multi-GPU sharding is a design note, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2302_12031_amd import ffrt
    from paper_2302_12031_amd import workloads as W

    torch.cuda.set_device(0)
    wl = make_workload(args)
    arch = {"none": None, "dense": ffrt.MLP_DENSE, "sparse": ffrt.MLP_SPARSE}[args.generator]
    rays = wl.num_rays
    kinds = {("collimated" if p.source.kind == 0 else "point") for p in wl.problems}
    stream = torch.cuda.Stream()
    shapes = tuple(int(x) for x in args.shapes.split(",")) if args.shapes else None
    R = timed_steps(ffrt, wl, args.steps, args.warmup, stream, arch=arch, shapes=shapes,
                    autotune=not args.no_autotune)
    plan, timed, st, T = R["plan"], R["timed"], R["st"], R["T"]
    ms_total, ms_step = R["ms_total"], R["ms_step"]
    stats = timed.decode_stats(st["stats"])
    loss_now = st["loss"].cpu().numpy()
    # the trace kernels alone, on the same stream, right after the timed region (HIP events in the library)
    with torch.cuda.stream(stream):
        scratch_irr = torch.empty_like(st["irr"])
        scratch_g = torch.empty_like(st["dLdP"])
        _, dLdI = timed.loss(st["irr"], T, stream=stream)
        fwd_ms, adj_ms = timed.time_kernels(st["Pz"], scratch_irr, dLdI, scratch_g, reps=args.steps,
                                            stream=stream)

    # ---- roofline of the dominant trace kernel; the forward's search steps from its own statistics (it starts
    # each Newton search at the previous ray's root), the adjoint's from a per-ray inspection
    iters = mean_search_steps(ffrt, wl, plan, st["Pz"])
    stt = timed.new_stats()
    timed.forward(st["Pz"], stats=stt)
    fstats = timed.decode_stats(stt)
    fwd_steps = [int(x) for x in fstats["n_search_steps"]]
    dom = "adjoint" if adj_ms >= fwd_ms else "forward"
    dom_ms = adj_ms if dom == "adjoint" else fwd_ms
    dom_flops, roots_reused = algorithmic_flops(wl, dom, iters, fwd_steps)
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            # HBM counters were taken on the exact-root, flat-entry kernels of the named workloads at their own sizes
            "traffic": None if (args.mesh or args.entry_freeform or args.rays_side)
            else _traffic(f"k_{dom}", args.workload),
            "kernel": f"k_{dom}", "kernel_ms": dom_ms, "flops_per_launch": dom_flops,
            "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
            "frac_of_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
            "forward_ms": fwd_ms, "adjoint_ms": adj_ms, "newton_iters_mean": iters,
            "forward_search_steps_per_ray": sum(fwd_steps) / max(1, int(fstats["n_traced"].sum())),
            "adjoint_reuses_exit_roots": roots_reused,
            "search_steps": "mesh cells visited" if args.mesh else "Newton iterations"}
    other = "forward" if dom == "adjoint" else "adjoint"
    other_flops, _ = algorithmic_flops(wl, other, iters, fwd_steps)
    other_ms = fwd_ms if other == "forward" else adj_ms
    roof[f"{other}_frac"] = other_flops / (other_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS
    roof["lds_atomics"] = lds_atomic_roofline(ffrt, wl, fstats, R["cfg"][0], fwd_ms, stream)

    generator = None
    if arch is not None:
        with torch.cuda.stream(stream):
            g_fwd, g_bwd, g_upd = timed.time_mlp(st, st["dLdP"], reps=args.steps, stream=stream)
        Ks = [p.lens.n_u * p.lens.n_v for p in wl.problems]
        Cs = [(2 * p.lens.p + 1) * (2 * p.lens.q + 1) for p in wl.problems]
        W_floats = sum(2 * K * K if arch == ffrt.MLP_DENSE else 2 * C * K for K, C in zip(Ks, Cs))
        n_par = timed.mlp_offsets(arch)[-1]
        groups = {"forward": (g_fwd, 4 * W_floats), "backprop": (g_bwd, 4 * W_floats), "update": (g_upd, 24 * n_par)}
        kern = {"forward": "k_mlp_layer1 + 2 x k_mlp_gemv" if arch == ffrt.MLP_DENSE else "k_smlp_forward",
                "backprop": "k_mlp_seed + 2 x k_mlp_gemv_t" if arch == ffrt.MLP_DENSE else "k_smlp_backprop",
                "update": "k_mlp_grad_adam" if arch == ffrt.MLP_DENSE else "k_smlp_update"}
        gname = max(groups, key=lambda k: groups[k][0])
        gms, gbytes = groups[gname]
        gach = gbytes / (gms * 1e-3) / 1e9
        groof = {"bound": "hbm", "achieved": gach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gach / PEAK_HBM_GBS,
                 "traffic": _traffic(kern[gname], f"{args.workload}-{args.generator}", "ffrt_mlp.hip"),
                 "kernel": kern[gname], "kernel_ms": gms, "bytes_per_launch": gbytes}
        generator = {"arch": args.generator, "parameters": n_par, "control_points": Ks,
                     "ms": {k: v[0] for k, v in groups.items()},
                     "bytes_per_launch": {k: v[1] for k, v in groups.items()}, "roofline": groof}
        if gms > dom_ms:
            roof = dict(groof, trace_kernels={"forward_ms": fwd_ms, "adjoint_ms": adj_ms,
                                              "alu_frac_of_dominant": achieved / PEAK_FP32_TFLOPS})

    out = {"metric": METRIC, "value": rays * args.steps / (ms_total * 1e-3), "unit": "rays/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": wl.name, "designs": len(wl.problems), "rays_per_step": rays,
                      "intersection": f"triangle mesh {args.mesh}x{args.mesh} per span" if args.mesh else "exact root",
                      "entry_face": "freeform" if args.entry_freeform else "flat",
                      "sources": sorted(kinds), "graph": f"{args.steps} captured steps",
                      "kernel_shapes": {"forward": R["cfg"][0], "adjoint": R["cfg"][1]}},
           "adam_steps_per_s": 1e3 / ms_step, "wall_s_timed": R["t_wall"],
           "loss_after": [float(x) for x in loss_now[:4]],
           "rays_hit_fraction": float(stats["n_hit"].sum()) / max(1, int(stats["n_traced"].sum())),
           "roofline": roof}
    if generator is not None:
        out["config"]["generator"] = args.generator
        out["generator"] = generator
    del R, timed, st

    # ---- finite-difference baseline on the same GPU (single-design workloads)
    if not args.no_fd and len(wl.problems) == 1 and arch is None:
        # at the initial design (the optimised one has rays parked on the screen edge by the target's dark
        # border, whose discrete flips within +-h make any finite difference ill-defined)
        out["fd"] = finite_differences(ffrt, W, wl, plan, T, ms_step, args.fd_oracle and not args.no_cpu)

    # ---- the same designs one plan (and one captured graph) each, launched one after another
    if args.compare_separate and len(wl.problems) > 1:
        sep_ms = separate_plans(ffrt, wl, stream, autotune=not args.no_autotune)
        out["separate_plans"] = {"designs": len(wl.problems), "ms_per_step_sum": sep_ms,
                                 "batched_ms_per_step": ms_step, "speedup_of_batching": sep_ms / ms_step,
                                 "rays_per_s_separate": rays / (sep_ms * 1e-3),
                                 "note": "each design autotuned in its own plan; graphs of 5 steps, run back to back"}

    # ---- secondary: the 64-design batch of uneven sizes (default workload only)
    if args.workload == "c4" and not (args.no_batch or args.rays_side or args.mesh or args.entry_freeform or arch):
        wb = W.c5()
        B = timed_steps(ffrt, wb, 20, 3, stream, autotune=not args.no_autotune, autotune_reps=3)
        sep_ms = separate_plans(ffrt, wb, stream, autotune=not args.no_autotune)
        out["batch"] = {"workload": wb.name, "designs": len(wb.problems), "rays_per_step": wb.num_rays,
                        "rays_per_s": wb.num_rays / (B["ms_step"] * 1e-3), "ms_per_step": B["ms_step"],
                        "design_steps_per_s": len(wb.problems) * 1e3 / B["ms_step"],
                        "separate_ms_per_step": sep_ms, "speedup_of_batching": sep_ms / B["ms_step"],
                        "kernel_shapes": {"forward": B["cfg"][0], "adjoint": B["cfg"][1]},
                        "note": "20 graph-captured steps of all designs in one plan, against every design in a "
                                "plan and a 5-step graph of its own (each autotuned), run back to back"}
        del B

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
