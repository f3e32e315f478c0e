"""Throughput of the multipatch RK4 wave step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched] [--precision mixed]

A step is one classic-RK4 step over every patch: four ghost fills (analytic and
periodic ghosts, global->local and local->global Lagrange interpolation with the
frame transform) and four fused RHS + stage-update launches, plus the end-of-step
cover flags and uncover fill.  Inputs start resident in HBM (exact initial data
computed on the device).  The timed region is exactly K steps between two
synchronisations, timed with HIP events on the library's stream.

Printed: one JSON line with the metric (live cell-updates per second), the
roofline figure of the dominant kernel (algorithmic bytes per launch divided by
its average duration, measured with HIP events in a separate eager pass), a
device-copy bandwidth measured in the same run, the batched mixed run against the
plain per-patch FP64 run (speed, accuracy against each other and against the
exact solution), the other mixed-precision variant, and the CPU oracle's rate on
a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_GFLOPS = 157300.0  # MI355X vector FP32 (dense)
FP64_PEAK_GFLOPS = 78600.0  # MI355X vector FP64
# Algorithmic bytes per live cell per stage kernel launch (five fields).
# FP64 path: stage 1 reads u, writes acc and v2; stages 2-3 read v_s, u, acc and
# write acc, v_{s+1}; stage 4 reads v4, acc and writes u (all 8-byte values).
# Mixed path, FP64 accumulator: stage 1 reads the FP32 copy of u (stencil input)
# and u, writes acc and v2; stages 2-3 read v_s, the FP32 copy of u and acc and
# write acc and v_{s+1}; stage 4 reads v4 and acc and writes u and its FP32 copy.
# Mixed path, FP32 increments: stage 1 reads the FP32 copy of u, writes the
# increment and v2; stages 2-3 read v_s, the copy of u and the increment and
# write the increment and v_{s+1}; stage 4 reads v4, the increment and u and
# writes u and its FP32 copy.
STAGE_BYTES = {"fp64": [120, 200, 200, 120], "mixed": [120, 140, 140, 120], "mixed_inc": [60, 100, 100, 140]}
DTYPE = {"fp64": "f64", "mixed": "f32+f64", "mixed_inc": "f32+f64"}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("pw_kernels.hip", "pw_internal.h", "pw_kernels.h"):
        with open(os.path.join(ROOT, "paper_2002_00088_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, precision, dominant):
    """HBM bytes per launch (FETCH + WRITE) of the dominant kernel from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, precision))
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("kernels", {}).get(dominant)


def g2l_points(cfg):
    """Ghost cells of the local patches filled from the global patch in one
    stage for the first state vector: the cells of the padded box outside the
    interior along a non-periodic axis."""
    tot = 0
    for p in cfg["patches"][1:]:
        if not (p["sv_mask"] & 1):
            continue
        full = inner = 1
        for a in range(3):
            full *= p["n"][a] + 6
            inner *= p["n"][a] + 6 if p["periodic"][a] else p["n"][a]
        tot += full - inner
    return tot


def make_config(name):
    from paper_2002_00088_amd import workloads as W
    if name == "batched":
        return W.batched(seed=4)
    if name == "two_patch":
        return W.two_patch(seed=2)
    if name == "spherical":
        return W.spherical(seed=3)
    if name == "periodic":
        return W.single_periodic(seed=1)
    if name == "multimethod":
        return W.multimethod(seed=5)
    if name == "three_topology":
        return W.three_topology()
    raise SystemExit("unknown workload " + name)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sample_config(name):
    """Bounded CPU sample of a workload: the same recipe at a smaller size (the
    batched workload scaled to a 96^3 global patch with 16-36 cells per local axis,
    about 5% of its cells), else the workload itself."""
    from paper_2002_00088_amd import workloads as W
    if name.startswith("batched"):
        return W.batched(seed=4, ng=96, nmin=16, nmax=36)
    return None


def cpu_baseline(cfg, reps=3):
    """The FP64 oracle as it stands, one RK4 step of a bounded sample of the
    workload, on one thread and on every host core (OpenMP), median of `reps`
    runs each, as live cell-updates per second."""
    from oracle.oracle import set_threads, world_from_config
    sample = cpu_sample_config(cfg["name"]) or cfg
    w = world_from_config(sample)
    w.init_exact(0.0)
    w.prepare()
    f, _ = w.flags()
    live = int((f == 0).sum()) + sum(int(p["n"][0] * p["n"][1] * p["n"][2]) for p in sample["patches"][1:])
    all_cores = set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    res = {}
    for th in (all_cores, 1):
        used = set_threads(th)
        secs = []
        for _ in range(reps):
            t0 = time.perf_counter()
            w.step(sample["dt"], 1)
            secs.append(time.perf_counter() - t0)
        res[used] = sorted(secs)[len(secs) // 2]
    set_threads(all_cores)
    w.close()
    return dict(value=live / res[all_cores], unit="cell-updates/s", cores=all_cores, kind="oracle",
                one_thread=dict(value=live / res[1], cores=1, median_s=round(res[1], 3)),
                median_s=round(res[all_cores], 3), reps=reps, cpu_model=cpu_model(),
                sample="one RK4 step of the %s workload (%d patches, %d live cells; the same recipe as %s at a "
                       "smaller size), FP64, median of %d" % (sample["name"], len(sample["patches"]), live,
                                                             cfg["name"], reps))


def copy_bandwidth(torch, stream, nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes on the same stream: (read + write) bytes
    per second, best of reps."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    best = 0.0
    with torch.cuda.stream(stream):
        dst.copy_(src)
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dst.copy_(src)
            e1.record(stream)
            e1.synchronize()
            best = max(best, 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    return best


def timed_steps(torch, ctx, stream, dt, steps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.rk4_step(dt, steps)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def errors_vs_exact(np, ctx, cfg):
    """Per field: max |u - exact| over live cells of every patch, relative to the
    largest |exact| there (the library's diagnostics, state vector 0)."""
    emax = np.zeros(5)
    umax = np.zeros(5)
    for pid in range(len(cfg["patches"])):
        d = ctx.diagnostics(pid, 0)
        emax = np.maximum(emax, d["err_max"])
        umax = np.maximum(umax, d["max"])
    return [float("%.3e" % x) for x in emax / np.maximum(umax, 1e-300)]


def compare_states(np, a_ctx, b_ctx, cfg):
    """Max and L2 differences of a against b over live cells of all patches,
    relative to b's largest magnitude (max) and norm (L2), per field."""
    f, _ = b_ctx.flags()
    maxabs = np.zeros(5)
    maxerr = np.zeros(5)
    l2 = np.zeros(5)
    nrm = np.zeros(5)
    for pid in range(len(cfg["patches"])):
        a, b = a_ctx.get_state(pid), b_ctx.get_state(pid)
        m = (f == 0) if pid == 0 else np.ones(a.shape[1:], dtype=bool)
        d = a[:, m] - b[:, m]
        maxabs = np.maximum(maxabs, np.abs(b[:, m]).max(axis=1))
        maxerr = np.maximum(maxerr, np.abs(d).max(axis=1))
        l2 += (d * d).sum(axis=1)
        nrm += (b[:, m] ** 2).sum(axis=1)
    return ([float("%.3e" % x) for x in maxerr / np.maximum(maxabs, 1e-300)],
            [float("%.3e" % x) for x in np.sqrt(l2 / np.maximum(nrm, 1e-300))])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "mixed_inc", "fp64"])
    ap.add_argument("--schedule", default="batched", choices=["batched", "per_patch"])
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default tuning")
    ap.add_argument("--torch-alloc", action="store_true",
                    help="the library allocates its device memory through torch's caching allocator")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one device copy of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2002_00088_amd import pw

    PREC = {"mixed": pw.PW_MIXED, "mixed_inc": pw.PW_MIXED_INC, "fp64": pw.PW_FP64}
    torch.cuda.set_device(0)
    cfg = make_config(args.workload)
    print("bench: workload %s, %d patches, precision %s, schedule %s" % (cfg["name"], len(cfg["patches"]),
                                                                         args.precision, args.schedule),
          file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    sched = pw.PW_SCHED_BATCHED if args.schedule == "batched" else pw.PW_SCHED_PER_PATCH
    ctx = pw.context_from_config(cfg, precision=PREC[args.precision], schedule=sched, use_graph=not args.no_graph,
                                 stream=stream.cuda_stream, torch_alloc=args.torch_alloc)
    dt = cfg["dt"]
    ctx.init_exact(0.0)
    if not args.no_autotune and sched == pw.PW_SCHED_BATCHED:
        # the library's autotuner on this workload (untimed; it advances the state,
        # so the initial data is set again afterwards)
        tuned = ctx.autotune(dt, 3)
        print("bench: autotuned %s" % tuned, file=sys.stderr, flush=True)
        ctx.init_exact(0.0)
    ctx.rk4_step(dt, args.warmup)
    stream.synchronize()
    live0 = ctx.live_cells()
    t_wall = time.perf_counter()
    ms = timed_steps(torch, ctx, stream, dt, args.steps) if args.steps > 0 else float("nan")
    t_wall = time.perf_counter() - t_wall
    live1 = ctx.live_cells()
    live = 0.5 * (live0 + live1)
    value = live * args.steps / (ms / 1e3) if args.steps > 0 else None
    print("bench: %.3f ms/step, %s cell-updates/s (wall %.3f s)" % (ms / max(1, args.steps),
                                                                     "%.3e" % value if value else "-", t_wall),
          file=sys.stderr, flush=True)

    # per-kernel-class durations (eager pass with HIP events on the same stream;
    # kernels one at a time)
    ctx.enable_timing(True)
    ctx.rk4_step(dt, args.timing_steps)
    kt = ctx.kernel_times()
    ctx.enable_timing(False)
    sb = STAGE_BYTES[args.precision]
    avg = {k: v[0] / max(1, v[1]) for k, v in kt.items()}
    nts = max(1, args.timing_steps)
    local_cells = sum(int(p["n"][0] * p["n"][1] * p["n"][2]) for p in cfg["patches"][1:])
    live_global = live - local_cells
    ty = "double, double, double" if args.precision == "fp64" else "float, float, float"
    tb = "double" if args.precision == "fp64" else "float"
    am = 1 if args.precision == "mixed_inc" else 0
    P = cfg["interp_points"][0]
    # GPU time per step of each single kernel (one kernel name in a profile) from
    # the eager pass: the interpolation kernels launch once per stage and state
    # vector, each global stage kernel once per step
    per_step = {}
    if kt["g2l"][1] > 0:
        per_step["g2l"] = kt["g2l"][0] / nts
    if kt["l2g"][1] > 0:
        per_step["l2g"] = kt["l2g"][0] / nts
    for st in range(4):
        per_step["gstage_s%d" % (st + 1)] = kt["gstage_s%d" % (st + 1)][0] / nts
    # the eager step: the top-level classes (the interpolation kernels and the
    # global stage launches are nested in the ghost-fill and stage classes)
    eager_step_ms = sum(v[0] for k, v in kt.items() if k not in ("g2l", "l2g") and not k.startswith("gstage")) / nts
    dom_key = max(per_step, key=per_step.get)
    copy_gbs = copy_bandwidth(torch, stream)
    tc_bytes = 8 if args.precision == "fp64" else 4

    gtile = ctx.tuning()["global_tile"]  # the global patch's tile shape (a template argument)

    def stage_roof(st):
        # the fused RHS + RK stage kernel over the global patch, stage st (HBM-bound)
        name = "k_stage<%s, %d, 0, true, %d, 0, %d>" % (ty, st, am, gtile)
        g_ms = avg["gstage_s%d" % (st + 1)]
        b = live_global * sb[st]
        a = b / (g_ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(a / HBM_PEAK_GBS, 4), "traffic": load_traffic(cfg["name"], args.precision, name),
                "kernel": name + " (RHS + RK stage %d, global patch)" % (st + 1), "avg_ms": round(g_ms, 5),
                "algorithmic_bytes_per_launch": int(b), "bytes_per_live_cell": sb[st], "live_cells": int(live_global),
                "eager_launches": int(kt["gstage_s%d" % (st + 1)][1]),
                "measured_copy_GBps": round(copy_gbs, 1), "frac_of_measured_copy": round(a / copy_gbs, 4)}

    def g2l_roof():
        # the global -> local interpolation kernel: 2 P^3 flops per field per ghost
        # point (a multiply and an add per tap), one state vector and one stage per
        # launch, against the FP32 vector peak; its taps come out of LDS
        name = "k_g2l_brick<%s, %s, %d>" % (tb, "double" if args.precision == "fp64" else "float", P)
        pts = g2l_points(cfg)
        g_ms = kt["g2l"][0] / kt["g2l"][1]
        flops = pts * 2 * 5 * P ** 3
        peak = FP64_PEAK_GFLOPS if args.precision == "fp64" else FP32_PEAK_GFLOPS
        a = flops / (g_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(a, 3), "peak": peak / 1e3, "unit": "TFLOP/s",
                "frac": round(a / (peak / 1e3), 4), "traffic": load_traffic(cfg["name"], args.precision, name),
                "kernel": name + " (global -> local interpolation)", "avg_ms": round(g_ms, 5),
                "points_per_launch": int(pts), "flops_per_point": 2 * 5 * P ** 3,
                "algorithmic_flops_per_launch": int(flops), "eager_launches": int(kt["g2l"][1]),
                "lds_bytes_per_point": 5 * P ** 3 * tc_bytes,
                "lds_read_TBps": round(pts * 5 * P ** 3 * tc_bytes / (g_ms * 1e-3) / 1e12, 2)}

    def l2g_roof():
        name = "k_l2g_bucket<%s, %s, %d>" % (tb, "double" if args.precision == "fp64" else "float", P)
        f, _ = ctx.flags()
        pts = int((f == 1).sum())
        g_ms = kt["l2g"][0] / kt["l2g"][1]
        flops = pts * 2 * 5 * P ** 3
        peak = FP64_PEAK_GFLOPS if args.precision == "fp64" else FP32_PEAK_GFLOPS
        a = flops / (g_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(a, 3), "peak": peak / 1e3, "unit": "TFLOP/s",
                "frac": round(a / (peak / 1e3), 4), "traffic": load_traffic(cfg["name"], args.precision, name),
                "kernel": name + " (local -> global interpolation)", "avg_ms": round(g_ms, 5),
                "points_per_launch": pts, "flops_per_point": 2 * 5 * P ** 3, "eager_launches": int(kt["l2g"][1])}

    if dom_key == "g2l":
        roofline = g2l_roof()
    elif dom_key == "l2g":
        roofline = l2g_roof()
    else:
        roofline = stage_roof(int(dom_key[-1]) - 1)
    tot_eager = eager_step_ms
    roofline["share_of_eager_step"] = round(per_step[dom_key] / tot_eager, 4)
    roofline["per_step_ms"] = round(per_step[dom_key], 5)
    # the HBM-bound stage kernel over the global patch at its step-average bytes
    # per live cell-stage (the four launches' mean duration)
    g_avg_ms = sum(avg["gstage_s%d" % (st + 1)] for st in range(4)) / 4
    b_avg = live_global * sum(sb) / 4
    a_avg = b_avg / (g_avg_ms * 1e-3) / 1e9
    roof_stage = {"bound": "hbm", "achieved": round(a_avg, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(a_avg / HBM_PEAK_GBS, 4), "kernel": "k_stage (global patch, mean of stages 1-4)",
                  "bytes_per_live_cell_stage": sum(sb) / 4, "avg_ms": round(g_avg_ms, 5),
                  "frac_of_measured_copy": round(a_avg / copy_gbs, 4),
                  "per_stage": [stage_roof(st) for st in range(4)]}
    roof_interp = {"g2l": g2l_roof() if kt["g2l"][1] > 0 else None, "l2g": l2g_roof() if kt["l2g"][1] > 0 else None}
    # all stage kernels of each stage (every patch), for reference
    stage_all = {"stage_s%d" % (s + 1): {"avg_ms": round(avg["stage_s%d" % (s + 1)], 5),
                                         "algorithmic_GBps": round(live * sb[s] / (avg["stage_s%d" % (s + 1)] * 1e-3) / 1e9, 1)}
                 for s in range(4)}
    step_bytes = live * sum(sb)
    step_ms = ms / max(1, args.steps)
    step_gbs = step_bytes / (step_ms * 1e-3) / 1e9
    kinds = {k: round(v, 5) for k, v in avg.items()}

    out = {"metric": "cell-updates/s per RK4 step (incl. ghost interp); HBM GB/s vs peak",
           "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[args.precision], "data": "synthetic",
           "config": {"workload": cfg["name"], "global_cells": cfg["patches"][0]["n"],
                      "local_patches": len(cfg["patches"]) - 1, "live_cells": int(live),
                      "precision": args.precision,
                      "schedule": args.schedule + ("" if args.no_graph or args.schedule != "batched" else "+graph"),
                      "dt": dt, "tuning": ctx.tuning(), "allocator": "torch" if args.torch_alloc else "hipMalloc"},
           "roofline": roofline,
           "step_hbm": {"achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(step_gbs / HBM_PEAK_GBS, 4), "target_frac": 0.6,
                        "bytes_per_live_cell_step": sum(sb), "measured_copy_GBps": round(copy_gbs, 1)},
           "roofline_stage": roof_stage,
           "roofline_interpatch": roof_interp,
           "stage_kernels_all_patches": stage_all,
           "kernel_per_step_ms": {k: round(v, 5) for k, v in per_step.items()},
           "kernel_avg_ms": kinds}
    n_total = args.warmup + args.steps + args.timing_steps

    if not args.no_compare and args.precision != "fp64":
        # plain per-patch FP64 on the same GPU, same number of steps; the accuracy
        # of the batched mixed run against it and of both against the exact solution
        ref = pw.context_from_config(cfg, precision=pw.PW_FP64, schedule=pw.PW_SCHED_PER_PATCH, use_graph=False,
                                     stream=stream.cuda_stream)
        ref.init_exact(0.0)
        ref.rk4_step(dt, args.warmup)
        stream.synchronize()
        ms_ref = timed_steps(torch, ref, stream, dt, args.steps)
        value_ref = ref.live_cells() * args.steps / (ms_ref / 1e3)
        ref.rk4_step(dt, args.timing_steps)
        emax, el2 = compare_states(np, ctx, ref, cfg)
        out["compare"] = {"per_patch_fp64": {"value": value_ref, "ms_per_step": ms_ref / args.steps,
                                             "max_rel_err_vs_exact": errors_vs_exact(np, ref, cfg)},
                          "batched_mixed_max_rel_err_vs_exact": errors_vs_exact(np, ctx, cfg),
                          "speedup_batched_mixed": value / value_ref,
                          "mixed_vs_fp64_max_rel_err": emax, "mixed_vs_fp64_l2_rel_err": el2,
                          "steps_compared": n_total}
        # the other mixed-precision variant, same steps, timed and compared the same way
        other = "mixed_inc" if args.precision == "mixed" else "mixed"
        var = pw.context_from_config(cfg, precision=PREC[other], schedule=sched, use_graph=not args.no_graph,
                                     stream=stream.cuda_stream)
        var.init_exact(0.0)
        if not args.no_autotune:
            var.autotune(dt, 3)
            var.init_exact(0.0)
        var.rk4_step(dt, args.warmup)
        stream.synchronize()
        ms_var = timed_steps(torch, var, stream, dt, args.steps)
        var.rk4_step(dt, args.timing_steps)
        vmax, vl2 = compare_states(np, var, ref, cfg)
        out["variant_" + other] = {"value": var.live_cells() * args.steps / (ms_var / 1e3),
                                   "ms_per_step": ms_var / args.steps,
                                   "stage_bytes_per_live_cell": STAGE_BYTES[other],
                                   "vs_fp64_max_rel_err": vmax, "vs_fp64_l2_rel_err": vl2,
                                   "max_rel_err_vs_exact": errors_vs_exact(np, var, cfg)}
        var.close()
        ref.close()
    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            dst.copy_(src)
        stream.synchronize()
        out["copy_probe_bytes"] = int(src.numel() * 4)
        del src, dst
    c = ctx.counters()
    out["counters"] = c
    ctx.close()
    if not args.no_cpu:
        print("bench: timing the CPU oracle on one step of the same workload", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
