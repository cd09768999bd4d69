#!/usr/bin/env python3
"""Benchmark: CTIS EM reconstruction of one synthetic frame on one MI355X.

One step = one full EM solve of the workload (the datacube reset to all ones,
then the configuration's iteration count of fused forward+ratio and
adjoint+update kernels), with the plan and the frame already resident in GPU
memory; by default the solve is captured once in a HIP graph and each step
replays it (``--launch stream`` launches the kernels one by one instead).  The JSON line reports EM iterations/s (the headline), voxel updates/s,
the roofline position of the dominant kernel (its average duration over a HIP
graph of back-to-back launches, HIP events around the replays), and the FP64
oracle's rate on the host cores over a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--config 3]

The default workload is the largest single-frame configuration (a = alpha =
128, w = 64, 1024 x 1024 FPA, 5 x 5 orders of 5 x 5 blobs, 200 iterations).
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EM iterations/s + voxel-updates/s vs HBM roofline; batched frames/s vs plain"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 157.3    # MI355X vector FP32 (counts packed FP32 FMA)
FP32_VALU_UNPACKED_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2006_01573_amd", "csrc", "kernels.hip")


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(config_id: int, kernel: str, choice: str | None = None, split: int = 1):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    counters, if they were taken on the current kernel source (and, for the
    batch, with the same launch choice and number of concurrent batches,
    whose launches of the kernel are then summed)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    w = d.get("workloads", {}).get(str(config_id), {})
    e = w.get(kernel)
    if not e or (choice is not None and (w.get("choice") != choice or int(w.get("split", 1)) != split)):
        return None
    return float(e["bytes_per_launch"])


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, g_host: np.ndarray, iters_per_step: int, seconds: float, solver: str = "em",
                 relax: float = 1.0):
    """The FP64 oracle (explicit H, OpenMP) on the host: iterations of the
    solver from all ones until `seconds` have passed, on all host cores and
    then on one core.  Assembly of the explicit H is excluded (and timed
    separately)."""
    import oracle
    progress("cpu baseline: assembling the explicit H")
    t0 = time.perf_counter()
    o = oracle.Oracle.from_case(case)
    t_asm = time.perf_counter() - t0

    def sample(budget):
        done, f = 0, None
        t1 = time.perf_counter()
        while True:
            if solver == "em":
                f = o.em(g_host, 1, f0=f)
            elif solver == "smart":
                f = o.smart(g_host, 1, f0=f)
            else:
                f = o.sart(g_host, 1, f0=f, relax=relax)
            done += 1
            el = time.perf_counter() - t1
            if el >= budget or done >= 100_000:
                return done, el

    all_threads = o.threads
    progress(f"cpu baseline: oracle EM on {all_threads} threads")
    done, el = sample(seconds)
    rate = done / el
    o.set_threads(1)
    progress("cpu baseline: oracle EM on 1 thread")
    done1, el1 = sample(seconds)
    o.close()
    rate1 = done1 / el1
    unit = "EM iterations/s" if solver == "em" else f"{solver.upper()} iterations/s"
    return {"value": rate, "unit": unit, "cores": all_threads, "kind": "oracle",
            "sample": f"{done} {solver.upper()} iterations of the same frame from all ones ({el:.1f} s, FP64 explicit "
                      f"sparse H, assembly of {t_asm:.1f} s excluded); one step of {iters_per_step} "
                      f"iterations would take {iters_per_step / rate:.2f} s",
            "host_cpu": host_cpu_model(),
            "one_core": {"value": rate1, "unit": unit, "cores": 1,
                         "sample": f"{done1} EM iterations ({el1:.1f} s)"}}


def region_arg(args, ctis):
    """--region RXxRY as the plan's region shape (0: the plan's choice);
    ValueError for a shape the plan does not take."""
    if not args.region:
        return 0
    try:
        shape = tuple(int(x) for x in args.region.lower().split("x"))
    except ValueError:
        shape = ()
    if shape not in ctis.REGION_SHAPES[1:]:
        raise ValueError(f"--region must be one of {', '.join(f'{a}x{b}' for a, b in ctis.REGION_SHAPES[1:])}")
    return shape


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4, 5],
                    help="1-3: one frame; 4: 64 uneven frames, batched vs sequential; "
                         "5: gradients of 10 unrolled EM iterations, 8 frames sharing one plan")
    ap.add_argument("--path", choices=["gather", "fourier"], default="gather",
                    help="gather: projections as gathers over the calibration nonzeros; fourier: the paper's "
                         "FFT form (configs 1-3)")
    ap.add_argument("--blob-radius", type=int, default=0, metavar="R",
                    help="with --path fourier: replace the configuration's calibration blobs by "
                         "(2R+1)^2 blobs (denser calibrations: the gather/Fourier crossover)")
    ap.add_argument("--c4-choice", default="", metavar="LABEL",
                    help="config 4: one batch with this launch choice (as the tuner labels it, e.g. "
                         "'tile 64x16 W4 adjoint W1 Bauto') instead of autotuning")
    ap.add_argument("--c4-split", type=int, default=1, metavar="N",
                    help="config 4 with --c4-choice: the frames in N batches of about equal work, run "
                         "concurrently on streams of their own (1..4; default 1: one batch)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="config 4: skip the 64 sequential single-frame solves")
    ap.add_argument("--solver", choices=["em", "smart", "sart"], default="em",
                    help="single-frame configs: the solver iterated (simultaneous MART or ART on the same "
                         "projections; default EM)")
    ap.add_argument("--relax", type=float, default=1.0, help="SART relaxation")
    ap.add_argument("--tile-path", action="store_true",
                    help="configs 1-3: EM on the tile path (64 x 16 FPA tiles read straight from f) instead "
                         "of the region path (16 x 16 regions read from a zero-bordered copy of f)")
    ap.add_argument("--region", default="", metavar="RXxRY",
                    help="configs 1-3: region shape of the region path (pixels along gamma x xi: 8x32, 16x16, "
                         "32x8, 16x8, 8x16 or 8x8; default the plan's choice)")
    ap.add_argument("--launch", choices=["graph", "stream"], default="graph",
                    help="graph: each step is one replay of a HIP graph holding the whole solve; "
                         "stream: the solve's kernels are launched one by one on the stream")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the path would shard by frame or by wavelength across GPUs, which is not built here.",
              file=sys.stderr)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        return 2
    # options checked before anything touches a device
    from paper_2006_01573_amd import ctis as _ctis, tune as _tune
    try:
        region_arg(args, _ctis)
    except ValueError as exc:
        print(f"bench.py: {exc}", file=sys.stderr)
        return 2
    if not 1 <= args.c4_split <= _tune.MAX_CONCURRENT or (args.c4_split > 1 and not args.c4_choice):
        print(f"bench.py: --c4-split takes 1..{_tune.MAX_CONCURRENT} and goes with --c4-choice", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    from paper_2006_01573_amd import ctis, workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}), flush=True)
        return 0
    if args.solver != "em":
        if args.config in (4, 5) or args.path == "fourier":
            print("bench.py: --solver applies to the single-frame gather configs 1-3", file=sys.stderr)
            return 2
        return bench_solver(args, torch, ctis, W, dev)
    if args.config == 4:
        return bench_batched(args, torch, ctis, W, dev)
    if args.config == 5:
        return bench_differentiable(args, torch, ctis, W, dev)
    if args.path == "fourier":
        return bench_fourier(args, torch, ctis, W, dev)
    case = W.make_case(args.config)
    cfg = case.cfg
    geo = case.geometry
    K = cfg.iters
    progress(f"workload {cfg.name}: plan")
    plan = ctis.Plan.from_case(case, tile_path=args.tile_path, region=region_arg(args, ctis))
    info = plan.info
    # the frame: Poisson noise on H f_true, formed with the library's own forward
    f_true = torch.from_numpy(case.f_true.astype(np.float32)).to(dev)
    clean = plan.forward(f_true).double().cpu().numpy()
    g_host = case.noisy(clean)
    g = torch.from_numpy(g_host).to(dev)
    f = torch.empty(plan.shape_f, dtype=torch.float32, device=dev)
    ws = plan.workspace()
    torch.cuda.synchronize()

    def solve():
        f.fill_(1.0)
        plan.em(g, K, f=f, workspace=ws)

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(run, steps):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), time.perf_counter() - w0

    def graph_of(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()                                   # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            fn()
        return gr

    solve_graph = graph_of(solve)
    step = solve_graph.replay if args.launch == "graph" else solve
    progress(f"warmup {args.warmup} steps ({args.launch} launch)")
    for _ in range(args.warmup):
        step()
    progress(f"timing {args.steps} steps of {K} EM iterations")
    ms, wall = timed(step, args.steps)
    sec = ms / 1e3
    it_s = args.steps * K / sec
    f_out = f.clone()
    if not torch.isfinite(f_out).all() or (f_out < 0).any():
        print("bench.py: EM produced a negative or non-finite value", file=sys.stderr)
        return 1
    other = solve if args.launch == "graph" else solve_graph.replay
    other_ms, _ = timed(other, args.steps)
    other_it_s = args.steps * K / (other_ms / 1e3)

    # per-kernel durations: an EM half launched back to back (the launches the
    # EM loop makes, on fixed inputs) inside one HIP graph of `reps` launches,
    # HIP events around its replays on the stream the graph runs on; the same
    # launches one by one on the stream for comparison.  On the region path
    # the forward half is two kernels (the padded copy of f, then the
    # projection) while the EM loop writes the padded copy once per solve, so
    # the forward kernel's duration there is the graph-launched EM iteration
    # less the back projection.
    progress("per-kernel timing pass")
    reps = 100
    f_in = f_out.clone()
    f_tmp = torch.empty_like(f_in)
    plan.em_forward_ratio(f_in, g, ws)
    avg, avg_stream = {}, {}
    halves = [("adjoint_update", lambda: plan.em_adjoint_update(ws, f_in, f_tmp))]
    if not info.em_region_path:
        halves.append(("forward_ratio", lambda: plan.em_forward_ratio(f_in, g, ws)))
    for name, launch in halves:
        def many(launch=launch):
            for _ in range(reps):
                launch()
        gr = graph_of(many)
        t, _ = timed(gr.replay, 5)
        avg[name] = t * 1e-3 / (5 * reps)
        t, _ = timed(many, 5)
        avg_stream[name] = t * 1e-3 / (5 * reps)
    if info.em_region_path:
        t_iter = (ms if args.launch == "graph" else other_ms) * 1e-3 / (args.steps * K)
        t_iter_stream = (other_ms if args.launch == "graph" else ms) * 1e-3 / (args.steps * K)
        avg["forward_ratio"] = t_iter - avg["adjoint_update"]
        avg_stream["forward_ratio"] = t_iter_stream - avg_stream["adjoint_update"]
    m, n_supp = info.m, info.n_support
    bytes_ = {"forward_ratio": 4 * (m + 2 * n_supp), "adjoint_update": 4 * (2 * m + n_supp)}
    flops_ = {k: 2 * info.ell * info.nnz for k in bytes_}
    dom = max(avg, key=avg.get)
    t_hbm = bytes_[dom] / (HBM_PEAK_GBS * 1e9)
    t_alu = flops_[dom] / (FP32_VALU_PEAK_TFLOPS * 1e12)
    traffic = measured_traffic(args.config, dom)
    if t_hbm >= t_alu:
        achieved = bytes_[dom] / avg[dom] / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    else:
        achieved = flops_[dom] / avg[dom] / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": traffic,
                "frac_of_unpacked_fp32": achieved / FP32_VALU_UNPACKED_TFLOPS}
    roof.update({"kernel": dom, "path": "region" if info.em_region_path else "tile",
                 "forward_timing": ("EM iteration less back projection (graph launched)" if info.em_region_path
                                    else "graph of back-to-back forward halves"),
                 "avg_launch_us": avg[dom] * 1e6,
                 "avg_launch_us_stream_launched": avg_stream[dom] * 1e6,
                 "algorithmic_bytes_per_launch": bytes_[dom], "algorithmic_flop_per_launch": flops_[dom],
                 "other_kernel": {k: {"avg_launch_us": avg[k] * 1e6,
                                      "avg_launch_us_stream_launched": avg_stream[k] * 1e6,
                                      "achieved_GBps": bytes_[k] / avg[k] / 1e9}
                                  for k in avg if k != dom}})

    line = {
        "metric": METRIC,
        "value": it_s,
        "unit": "EM iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "a": geo.a, "alpha": geo.alpha, "w": geo.w,
                   "gamma": geo.gamma, "xi": geo.xi, "m": m, "n": geo.n, "n_support": n_supp,
                   "nnz": info.nnz, "box": info.box, "em_iters_per_step": K,
                   "forward_path": "region" if info.em_region_path else "tile",
                   **({"region": f"{info.region_fast}x{info.region_slow}"} if info.em_region_path else {}),
                   "forward_executed_madds_over_method": ((info.region_forward_madds if info.em_region_path
                                                           else info.tile_forward_madds) / info.method_madds),
                   "start": "all ones", "noise": f"Poisson, {cfg.noise} {cfg.photons:g}"},
        "voxel_updates_per_s": it_s * m,
        "frames_per_s": args.steps / sec,
        "wall_s": wall,
        "launch": args.launch,
        ("stream_launch_em_iters_per_s" if args.launch == "graph" else "graph_launch_em_iters_per_s"): other_it_s,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, g_host, K, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    plan.close()
    return 0


def bench_solver(args, torch, ctis, W, dev) -> int:
    """The single-frame solve with simultaneous MART or ART (ctis_solve_iterate)
    in place of EM: the same projections with other epilogues, the same
    iteration count, graph-launched.  The roofline position is that of one
    iteration (forward and back projection together), from the graph-launched
    solve's time per iteration."""
    case = W.make_case(args.config)
    cfg, geo, K = case.cfg, case.geometry, case.cfg.iters
    progress(f"workload {cfg.name}: plan ({args.solver})")
    plan = ctis.Plan.from_case(case, tile_path=args.tile_path, region=region_arg(args, ctis))
    info = plan.info
    clean = plan.forward(torch.from_numpy(case.f_true.astype(np.float32)).to(dev)).double().cpu().numpy()
    g_host = case.noisy(clean)
    g = torch.from_numpy(g_host).to(dev)
    f = torch.empty(plan.shape_f, dtype=torch.float32, device=dev)
    ws = plan.solve_workspace()

    def solve():
        f.fill_(1.0)
        plan.solve(g, K, solver=args.solver, relax=args.relax, f=f, workspace=ws)

    gr = _graph_of(torch, solve)
    for _ in range(args.warmup):
        gr.replay()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        gr.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    if not torch.isfinite(f).all() or (f < 0).any():
        print("bench.py: the solve produced a negative or non-finite value", file=sys.stderr)
        return 1
    it_s = args.steps * K / (ms / 1e3)
    t_it = 1.0 / it_s
    m, n_supp = info.m, info.n_support
    bytes_it = 4 * (m + 2 * n_supp) + 4 * (2 * m + n_supp)
    flops_it = 4 * info.ell * info.nnz
    if bytes_it / (HBM_PEAK_GBS * 1e9) >= flops_it / (FP32_VALU_PEAK_TFLOPS * 1e12):
        achieved = bytes_it / t_it / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    else:
        achieved = flops_it / t_it / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": None,
                "frac_of_unpacked_fp32": achieved / FP32_VALU_UNPACKED_TFLOPS}
    roof.update({"kernel": "one iteration (forward and back projection, graph launched)",
                 "path": "region" if info.em_region_path else "tile", "avg_iteration_us": t_it * 1e6,
                 "algorithmic_bytes_per_iteration": bytes_it, "algorithmic_flop_per_iteration": flops_it})
    line = {
        "metric": METRIC,
        "value": it_s,
        "unit": f"{args.solver.upper()} iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name + f" ({args.solver.upper()} in place of EM)", "solver": args.solver,
                   "relax": args.relax if args.solver == "sart" else None, "iters_per_step": K, "m": m, "n": geo.n,
                   "forward_path": "region" if info.em_region_path else "tile",
                   **({"region": f"{info.region_fast}x{info.region_slow}"} if info.em_region_path else {})},
        "voxel_updates_per_s": it_s * m,
        "wall_s": wall,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, g_host, K, args.cpu_seconds, args.solver, args.relax)
    print(json.dumps(line), flush=True)
    plan.close()
    return 0


def bench_batched(args, torch, ctis, W, dev) -> int:
    """64 uneven frames (a = alpha in {32, 48, 64}, w in {16, 32}, FPA 256 or
    512), 50 EM iterations each: the autotuned batch (one launch per kernel per
    iteration for all frames, the iteration loop captured in a HIP graph)
    against 64 sequential single-frame solves."""
    from paper_2006_01573_amd import tune
    cfgs = W.batched_configs(64)
    K = cfgs[0].iters
    progress("c4: 64 plans and frames")
    cases = [W.make_case(4, frame=k, cfg=c) for k, c in enumerate(cfgs)]
    plans = [ctis.Plan.from_case(c) for c in cases]
    images = []
    for c, p in zip(cases, plans):
        clean = p.forward(torch.from_numpy(c.f_true.astype(np.float32)).to(dev)).double().cpu().numpy()
        images.append(c.noisy(clean))
    if args.c4_choice:
        progress(f"c4: the given launch choice ({args.c4_choice}), {args.c4_split} batch(es)")
        tuned = None
        b = tune.fixed_frames(cases, tune.Choice.parse(args.c4_choice), split=args.c4_split)
    else:
        progress("c4: autotuning per frame shape")
        tuned = tune.autotune_frames(cases, images, iters=4, reps=3)
        b = tuned.batch
    g_all = b.pack_g(images)
    ws = b.workspace()
    f_all = torch.ones(b.m_total, dtype=torch.float32, device=dev)
    # capture the whole solve (reset + K iterations) once, replay it per step
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        f_all.fill_(1.0)
        b.em(g_all, K, f_all=f_all, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        f_all.fill_(1.0)
        b.em(g_all, K, f_all=f_all, workspace=ws)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    progress(f"c4: timing {args.steps} batched solves")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    batched_fps = 64 * args.steps / (ms / 1e3)
    out = f_all.clone()
    if not torch.isfinite(out).all() or (out < 0).any():
        print("bench.py: EM produced a negative or non-finite value", file=sys.stderr)
        return 1
    seq = {}
    if not args.no_sequential:
        # sequential: 64 plain single-frame solves per step
        progress("c4: timing sequential single-frame solves")
        gs = [torch.from_numpy(im).to(dev) for im in images]
        fs = [torch.empty(p.shape_f, dtype=torch.float32, device=dev) for p in plans]
        wss = [p.workspace() for p in plans]

        def seq_step():
            for p, gk, fk, wk in zip(plans, gs, fs, wss):
                fk.fill_(1.0)
                p.em(gk, K, f=fk, workspace=wk)

        seq_step()
        torch.cuda.synchronize()
        seq_steps = max(1, args.steps // 2)
        e0.record()
        for _ in range(seq_steps):
            seq_step()
        e1.record()
        torch.cuda.synchronize()
        seq_fps = 64 * seq_steps / (e0.elapsed_time(e1) / 1e3)
        # the same 64 solves, each frame's solve replayed from its own HIP graph
        progress("c4: timing sequential single-frame solves from HIP graphs")
        graphs = []
        for p, gk, fk, wk in zip(plans, gs, fs, wss):
            def one(p=p, gk=gk, fk=fk, wk=wk):
                fk.fill_(1.0)
                p.em(gk, K, f=fk, workspace=wk)
            graphs.append(_graph_of(torch, one))
        e0.record()
        for _ in range(seq_steps):
            for gr_k in graphs:
                gr_k.replay()
        e1.record()
        torch.cuda.synchronize()
        seq_graph_fps = 64 * seq_steps / (e0.elapsed_time(e1) / 1e3)
        seq = {"sequential_frames_per_s": seq_fps, "batched_vs_sequential": batched_fps / seq_fps,
               "sequential_graph_frames_per_s": seq_graph_fps,
               "batched_vs_sequential_graph": batched_fps / seq_graph_fps}
    # per-kernel durations: each batch's EM halves launched `reps` times back
    # to back inside a HIP graph (own workspace per batch, fixed inputs), HIP
    # events around 5 replays on the graph's stream.  On the region path the
    # forward half also writes the padded copy of f, which the EM loop does
    # once per solve, so there the forward's duration is the batch's
    # graph-launched EM iteration (`reps` iterations in one call) less its
    # back projection.
    progress("c4: per-kernel timing pass")
    reps = 20
    infos = [p.info for p in plans]
    m_all = sum(i.m for i in infos)
    nsup = sum(i.n_support for i in infos)
    flops = sum(2 * i.ell * i.nnz for i in infos)
    parts = b.parts(g_all, f_all)
    avg = {"forward_ratio": 0.0, "adjoint_update": 0.0}

    def graph_time(fn):
        gr = _graph_of(torch, fn)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            gr.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / (5 * reps)

    region_parts = 0
    for bk, gk, fk in parts:
        wk = bk.workspace()
        f_in = fk.clone()
        f_tmp = torch.empty_like(f_in)
        bk.em_forward_ratio(f_in, gk, wk)
        t_adj = graph_time(lambda: [bk.em_adjoint_update(wk, f_in, f_tmp) for _ in range(reps)])
        if bk.info["em_region_path"]:
            region_parts += 1
            f_it = f_in.clone()
            t_fwd = graph_time(lambda: bk.em(gk, reps, f_all=f_it, workspace=wk)) - t_adj
        else:
            t_fwd = graph_time(lambda: [bk.em_forward_ratio(f_in, gk, wk) for _ in range(reps)])
        avg["adjoint_update"] += t_adj
        avg["forward_ratio"] += t_fwd
    it_s_total = avg["forward_ratio"] + avg["adjoint_update"]
    bytes_ = {"forward_ratio": 4 * (m_all + 2 * nsup), "adjoint_update": 4 * (2 * m_all + nsup)}
    dom = max(avg, key=avg.get)
    t_hbm = bytes_[dom] / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (FP32_VALU_PEAK_TFLOPS * 1e12)
    groups = b.report()
    # counters recorded for this launch choice and split (bytes of all of an
    # iteration's launches of the kernel: one per batch)
    same = len({g["choice"] for g in groups}) == 1 and (len(groups) == 1 or b.concurrent)
    traffic = measured_traffic(4, dom, groups[0]["choice"], len(groups)) if same else None
    if t_hbm >= t_alu:
        achieved = bytes_[dom] / avg[dom] / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    else:
        achieved = flops / avg[dom] / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": traffic,
                "frac_of_unpacked_fp32": achieved / FP32_VALU_UNPACKED_TFLOPS}
    roof.update({"kernel": dom + " (all 64 frames)", "launches_per_iteration": len(parts),
                 "forward_timing": ("EM iteration less back projection (graph launched)" if region_parts
                                    else "graph of back-to-back forward halves"),
                 "avg_launch_us": avg[dom] * 1e6,
                 "algorithmic_bytes_per_launch": bytes_[dom], "algorithmic_flop_per_launch": flops,
                 "other_kernel": {k: {"avg_launch_us": avg[k] * 1e6, "achieved_GBps": bytes_[k] / avg[k] / 1e9,
                                      "achieved_TFLOPs": flops / avg[k] / 1e12}
                                  for k in avg if k != dom},
                 "hbm_GBps_per_iteration": (bytes_["forward_ratio"] + bytes_["adjoint_update"]) / it_s_total / 1e9,
                 # the same bytes over the solve's own time per iteration (graph-launched, every batch of
                 # the arrangement; concurrent batches overlap their kernels, which the per-kernel times
                 # above, taken one batch at a time, do not show)
                 "hbm_GBps_per_solve_iteration": (bytes_["forward_ratio"] + bytes_["adjoint_update"])
                 / (ms * 1e-3 / (args.steps * K)) / 1e9})
    if tuned is not None:
        tuned_info = {"arrangement": tuned.arrangement, "batches": b.report(), "uniform_choice": tuned.uniform,
                      "ms_per_iter_of_arrangements": tuned.ms_per_iter, "per_shape": tuned.classes,
                      "candidates_timed": len(tuned.table)}
    else:
        tuned_info = {"arrangement": "given" + (f", {len(b.groups)} concurrent" if b.concurrent else ""),
                      "batches": b.report()}
    line = {
        "metric": METRIC,
        "value": batched_fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c4 64 uneven frames, a=alpha in {32,48,64}, w in {16,32}, FPA 256/512, "
                               "3x3 orders, 50 EM iterations each, one step = all 64 frames",
                   "frames": 64, "em_iters": K, "m_total": m_all, "n_support_total": nsup,
                   "tuned": tuned_info},
        **seq,
        "em_iteration_all_frames_us": ms * 1e3 / (args.steps * K),
        "roofline": roof,
    }
    print(json.dumps(line), flush=True)
    return 0


def _graph_of(torch, fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        fn()
    return gr


def bench_fourier(args, torch, ctis, W, dev) -> int:
    """The same single-frame EM solve through the Fourier (WBH) projections:
    per iteration w/2 + 1 forward and w/2 + 1 inverse complex FFTs of length
    n (two FFT passes each), with the gather path's rate beside it."""
    if args.blob_radius > 0:
        base = W.CONFIGS[args.config]
        R = args.blob_radius
        cfg0 = W.Config(f"{base.name} with {2 * R + 1}x{2 * R + 1} blobs", base.geometry,
                        W.KernelModel(base.kernel.orders, R, 0.4 * R + 0.4, base.kernel.dispersion),
                        iters=base.iters, noise=base.noise, photons=base.photons)
        case = W.make_case(args.config, cfg=cfg0)
    else:
        case = W.make_case(args.config)
    cfg, geo, K = case.cfg, case.geometry, case.cfg.iters
    progress(f"fourier {cfg.name}: plan and spectra")
    plan = ctis.Plan.from_case(case)
    F = ctis.Fourier(plan)
    clean = plan.forward(torch.from_numpy(case.f_true.astype(np.float32)).to(dev)).double().cpu().numpy()
    g = torch.from_numpy(case.noisy(clean)).to(dev)
    f = torch.empty(plan.shape_f, dtype=torch.float32, device=dev)
    ws = F.workspace()
    wsg = plan.workspace()

    def solve():
        f.fill_(1.0)
        F.em(g, K, f=f, workspace=ws)

    def solve_gather():
        f.fill_(1.0)
        plan.em(g, K, f=f, workspace=wsg)

    gr = _graph_of(torch, solve)
    for _ in range(args.warmup):
        gr.replay()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        gr.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    it_s = args.steps * K / (ms / 1e3)
    if not torch.isfinite(f).all():
        print("bench.py: Fourier EM produced a non-finite value", file=sys.stderr)
        return 1
    grg = _graph_of(torch, solve_gather)
    grg.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        grg.replay()
    e1.record()
    torch.cuda.synchronize()
    gather_it_s = args.steps * K / (e0.elapsed_time(e1) / 1e3)
    P, N, m = F.info["pairs"], geo.n, geo.m
    # algorithmic bytes of one Fourier EM iteration (FFT passes read and write n
    # complex values; the fused loads and stores add f, g, u and the spectra):
    # 12 m + 72 P n + 52 n
    bytes_it = 12 * m + 72 * P * N + 52 * N
    it_us = ms * 1e3 / (args.steps * K)
    achieved = bytes_it / (it_us * 1e-6) / 1e9
    line = {
        "metric": METRIC,
        "value": it_s,
        "unit": "EM iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name + " (Fourier projections)", "n": N, "fft": f"{F.info['n1']}x{F.info['n2']}",
                   "pairs": P, "em_iters_per_step": K, "nnz_per_wavelength": plan.info.nnz // geo.w},
        "voxel_updates_per_s": it_s * m,
        "gather_path_em_iters_per_s": gather_it_s,
        "fourier_vs_gather": it_s / gather_it_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "one Fourier EM iteration (8 FFT pass launches)", "avg_iteration_us": it_us,
                     "algorithmic_bytes_per_iteration": bytes_it},
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_differentiable(args, torch, ctis, W, dev) -> int:
    """8 frames of the c2 shape sharing one calibration plan; one step = the
    loss sum ||f^(K+1) - f_true||^2 of K = 10 unrolled EM iterations and its
    gradients with respect to f0 and every calibration value (set the
    values, K checkpointed EM iterations, K derivative calls)."""
    from paper_2006_01573_amd.autodiff import unrolled_em
    K = 10
    cases = W.differentiable_cases(8, iters=K)
    c0 = cases[0]
    nf = len(cases)
    progress(f"c5: plan and {nf} frames")
    plan = ctis.Plan.from_case(c0, keep_zeros=True)
    # the checkpointed forward runs one EM iteration per call: the tile path,
    # which needs no padded copy of f per call
    b = ctis.Batch([plan] * nf, tile_path=True)
    images = []
    for c in cases:
        clean = plan.forward(torch.from_numpy(c.f_true.astype(np.float32)).to(dev)).double().cpu().numpy()
        images.append(c.noisy(clean))
    g_all = b.pack_g(images)
    target = torch.from_numpy(np.concatenate([c.f_true.ravel() for c in cases]).astype(np.float32)).to(dev)
    f0 = torch.ones(int(b.f_offsets[-1]), dtype=torch.float32, device=dev, requires_grad=True)
    v = torch.from_numpy(c0.value.astype(np.float32)).to(dev).requires_grad_(True)

    def step():
        f0.grad = None
        v.grad = None
        fK = unrolled_em(b, g_all, f0, K, values=v)
        loss = ((fK - target) ** 2).sum()
        loss.backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    progress(f"c5: timing {args.steps} gradient steps")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        loss = step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    if not (torch.isfinite(f0.grad).all() and torch.isfinite(v.grad).all()):
        print("bench.py: non-finite gradient", file=sys.stderr)
        return 1
    # the pieces: one batched EM iteration and one batched derivative call
    ws = b.vjp_workspace()
    f_all = torch.ones_like(target)
    y = torch.randn_like(target)
    dv = torch.zeros(b.info["n_entries"], dtype=torch.float32, device=dev)
    reps = 20
    b.em(g_all, 1, f_all=f_all, workspace=ws)
    e0.record()
    for _ in range(reps):
        b.em(g_all, 1, f_all=f_all, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    em_us = e0.elapsed_time(e1) / reps * 1e3
    f_in = f_all.clone()
    b.em_vjp(g_all, f_in, y, df_all=y, dvalues=dv, accumulate=True, workspace=ws)
    e0.record()
    for _ in range(reps):
        b.em_vjp(g_all, f_in, y, df_all=y, dvalues=dv, accumulate=True, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    vjp_us = e0.elapsed_time(e1) / reps * 1e3
    inf = plan.info
    m_all, nsup = nf * inf.m, nf * inf.n_support
    # algorithmic bytes of one derivative call: forward+ratio (f, g, u), back
    # projection (u; y, f in; zeta, b out), forward of b (b, g, u; e out), back
    # projection (e; y, zeta in; df out), value partials (u, e, b, f)
    bytes_vjp = 4 * (11 * m_all + 9 * nsup)
    achieved = bytes_vjp / (vjp_us * 1e-6) / 1e9
    line = {
        "metric": METRIC,
        "value": nf * args.steps / (ms / 1e3),
        "unit": "differentiated frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c5 8 frames a=alpha=64 w=32 FPA512 sharing one calibration plan, loss "
                               "||f^(11) - f_true||^2 after 10 unrolled EM iterations, gradients w.r.t. f0 "
                               "and all calibration values; one step = forward + backward",
                   "frames": nf, "em_iters": K, "m_total": m_all, "n_entries": int(b.info["n_entries"])},
        "loss": float(loss.item()),
        "wall_s": wall,
        "em_iteration_all_frames_us": em_us,
        "vjp_call_all_frames_us": vjp_us,
        "vjp_vs_em_iteration": vjp_us / em_us,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(5, "derivative_call"),
                     "kernel": "one derivative call of all frames (4 projections + value partials + sums)",
                     "algorithmic_bytes_per_call": bytes_vjp},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
