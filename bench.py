"""Throughput of the Teukolsky Lax-Wendroff step on one MI355X.

A "step" is one full time step (stage lw1 then lw2) of the headline workload:
s = -2, m = 2, a/M = 0.9 on 4096 r* x 128 theta, r* in [-200, 800] M, FP64,
10,000 steps (at CFL 0.15: at the stated 0.5 the run is unstable; the cost
per update does not depend on the time step).  value = grid-point updates per
second (n_r * n_theta per step) over exactly --steps timed steps, inputs
resident in HBM; the launch shape is picked by the autotuner before timing.  The same JSON line
carries the double-double and quad-double workloads, the batched-vs-loop
comparison, the roofline of the step kernel and the oracle timed on the host
cores.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector

# Counter-derived figures, valid only for the launch shapes and kernel sources
# they were taken with (`source` is kernel_source_digest() of those sources;
# for other sources they are reported as null).  profiles/lw_wide_fp64_4096x128.md
# and profiles/lw_wide_valu_f64_counts.md give the rocprofv3 commands (--pmc on
# paper_1006_0663_amd/profile_step.py, one MI355X).
#  traffic: HBM bytes per launch of the headline kernel, FETCH_SIZE and
#    WRITE_SIZE in KiB; a 256 MiB device copy reads FETCH_SIZE 131,093 KiB
#    (scale 2.0) and WRITE_SIZE 262,144 KiB (scale 1.0).  Key: (sweep,
#    segcols, block, steps per launch); the slab sweep's launch runs the
#    whole timed call (20 steps in the default run).
#  fp64_flops_hw: FP64 operations per update as the hardware counts them
#    (SQ_INSTS_VALU_FLOPS_FP64 = 2 FMA + ADD + MUL wave instructions, x 64
#    lanes, per launch, over the updates of that launch): unlike the operation
#    tally of opcount.py this includes the halo columns each segment
#    recomputes and lanes whose results are discarded.  Key: (workload,
#    sweep, segcols, block, steps per launch).
#  fp64_mix: FP64 VALU lane-instructions per update (ADD, MUL, FMA, TRANS),
#    from SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 in the same way.  Key as
#    fp64_flops_hw.
MEASURED = {
    "source": "0631f1e0dfb0", "fetch_scale": 2.0, "write_scale": 1.0,
    "traffic": {(3, 16, 1024, 20): (45799.6, 92557.5)},
    "fp64_flops_hw": {
        ("fp64-4096x128", 3, 16, 1024, 1): 256.0,
        ("fp64-256x32", 1, 4, 512, 4): 959.5,
        ("dd-256x32", 1, 2, 256, 2): 5066.0,
        ("dd-1024x64", 3, 4, 256, 1): 1604.0,
        ("dd-4096x128", 1, 8, 256, 1): 1829.8,
        ("qd-2048x64", 3, 8, 512, 1): 13324.0,
        ("qd-4096x128", 1, 16, 256, 1): 14260.5,
    },
    "fp64_mix": {
        ("fp64-4096x128", 3, 16, 1024, 1): (28.0, 42.0, 92.0, 2.0),
        ("fp64-256x32", 1, 4, 512, 4): (101.5, 153.8, 348.5, 7.2),
        ("dd-256x32", 1, 2, 256, 2): (3074.0, 336.0, 828.0, 0.0),
        ("dd-1024x64", 3, 4, 256, 1): (992.0, 108.0, 252.0, 0.0),
        ("dd-4096x128", 1, 8, 256, 1): (1121.9, 123.0, 292.4, 0.0),
        ("qd-2048x64", 3, 8, 512, 1): (11176.0, 636.0, 756.0, 0.0),
        ("qd-4096x128", 1, 16, 256, 1): (11942.7, 684.6, 816.6, 0.0),
    },
}


def measured(table, key):
    if kernel_source_digest() != MEASURED["source"]:
        return None
    return MEASURED[table].get(tuple(key))


def kernel_source_digest():
    """Digest of every library source (kernels, launch code, header)."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_1006_0663_amd", "csrc")
    files = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))] + [os.path.join(ROOT, "include", "teuk.h")]
    for path in files:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode() + b"\0" + fh.read())
    return h.hexdigest()[:12]


def _torch():
    import torch
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    return torch


SWEEP_NAMES = ["segment", "wide", "wide2", "slab"]
SLAB = 3
SLAB_MAX_STEPS = 4096           # steps of one slab launch at most (the library's limit)


def launch_steps(shape, steps):
    """Steps one launch of this shape advances in a run of `steps`: the fused
    count, or for the persistent slab sweep the whole call (up to its limit)."""
    return min(steps, SLAB_MAX_STEPS) if shape[0] == SLAB else shape[3]


def kernel_name(shape, ns, nth):
    if shape[0] == SLAB:       # block, columns per lane = segcols / (block / n_theta)
        return "lw_slab_kernel<%d,%d> (persistent, %d steps per launch)" % (shape[2], shape[1] * nth // shape[2], ns)
    return (["lw_step_kernel<double>", "lw_wide_kernel<double,run 1>", "lw_wide_kernel<double,run 2>"][shape[0]]
            + ("" if ns == 1 else " (%d steps per launch)" % ns))


def graph_length(graph, steps):
    """Steps per captured graph for a timed run of `steps`: the requested
    length when the run holds at least one such graph, else no graph (a run
    shorter than one graph is a handful of launches, which a graph replay does
    not make faster: measured on the headline, 20 steps took 12.2 us per step
    as plain launches and 12.5 as one replay)."""
    return graph if graph and steps >= graph else 0


def time_single(T, w, fields, steps, warmup, graph, tile, torch, stream, log=None, fixed_shape=None,
                round_trip=False):
    """Time `steps` steps after `warmup` untimed ones, in the autotuned (or
    given) launch shape, with HIP graphs of graph_length(graph, steps) steps
    captured before the warm-up.  Returns (ms, wall s, fields finite, shape,
    graph replays in the timed region, steps those replays covered)."""
    from paper_1006_0663_amd import autotune
    g = T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass, w.angular_order)
    h = T.Teuk(w.s, w.m, w.a_over_M, g, w.words)
    h.set_stream(stream.cuda_stream)
    h.set_initial(*fields)
    glen = graph_length(graph, steps)
    if glen:
        h.use_graph(glen)           # before tuning: candidates are timed as they will run
    if fixed_shape:
        autotune.apply(h, fixed_shape)
        shape = tuple(fixed_shape) + (1,) * (4 - len(fixed_shape))
    elif tile:
        h.set_launch(tile, 0)
        shape = (h.sweep, tile, 0, 1)
    else:
        shape = autotune.tune(h, w.words, [(w.n_r, w.n_theta)], torch, stream, steps=max(20, 2 * glen))[:4]
    if round_trip:
        h.set_host_round_trip(True)
    h.prepare_graph()
    h.set_initial(*fields)
    with torch.cuda.stream(stream):
        h.step(warmup)
        torch.cuda.synchronize()
        r0 = h.graph_replays
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        h.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    replays = h.graph_replays - r0
    gsteps = max(1, glen // shape[3]) * shape[3] if glen else 0
    finite = h.check_finite()
    h.close()
    return ms, wall, finite, shape, replays, replays * gsteps


def cpu_baseline(w, seconds_target=22.0, single_core_seconds=6.0):
    """The oracle (C fixed-point engine, all host cores) on a radial slab of the
    headline workload: 512 r* nodes around the pulse x all theta rows."""
    from paper_1006_0663_amd import inputs
    from oracle import engine, problem
    nslab = 512
    full = inputs.initial_fields(w)
    peak = int(abs(full[0][..., 0]).sum(axis=0).argmax())
    i0 = max(0, min(w.n_r - nslab, peak - nslab // 2))
    h = (w.rstar_max - w.rstar_min) / (w.n_r - 1)
    # same spacing and time step as the full grid: dt = cfl*min(h, dtheta)
    slab = problem.Problem(w.s, w.m, w.a_over_M, nslab, w.n_theta, w.rstar_min + i0 * h,
                           w.rstar_min + (i0 + nslab - 1) * h, w.cfl)
    cores = os.cpu_count() or 1
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    tab = problem.build_tables(slab, processes=min(cores, 16))
    FT = engine.tables_to_fixed(tab, processes=min(cores, 16))
    u = engine.fields_to_fixed([f[:, i0:i0 + nslab] for f in full])
    engine.run_fixed(FT, nslab, w.n_theta, u, 1, threads=cores)      # thread start-up
    t0 = time.perf_counter()
    engine.run_fixed(FT, nslab, w.n_theta, u, 3, threads=cores)
    one = (time.perf_counter() - t0) / 3
    nsteps = max(1, int(seconds_target / max(one, 1e-3)))
    t0 = time.perf_counter()
    engine.run_fixed(FT, nslab, w.n_theta, u, nsteps, threads=cores)
    dt = time.perf_counter() - t0
    cores = engine.threads_in_use()
    # one core, as the paper's CPU baseline ran: a shorter sample of the same slab
    t0 = time.perf_counter()
    engine.run_fixed(FT, nslab, w.n_theta, u, 1, threads=1)
    one1 = time.perf_counter() - t0
    n1 = max(1, int(single_core_seconds / max(one1, 1e-3)))
    t0 = time.perf_counter()
    engine.run_fixed(FT, nslab, w.n_theta, u, n1, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": nslab * w.n_theta * nsteps / dt, "unit": "grid-point updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d steps of a %d x %d r*-slab (nodes %d..%d) of the headline grid, 384-bit fixed point, %.1f s"
                      % (nsteps, nslab, w.n_theta, i0, i0 + nslab - 1, dt),
            "cpu_model": _cpu_model(),
            "single_core": {"value": nslab * w.n_theta * n1 / dt1, "unit": "grid-point updates/s", "cores": 1,
                            "sample": "%d steps of the same slab on one thread, %.1f s" % (n1, dt1),
                            "threads_checked": engine.threads_in_use()}}


def issue_ceiling(name, shape, pct_hw):
    """Share of the FP64 peak a kernel could reach with every VALU issue slot
    holding one of its FP64 instructions (the peak counts an FMA as two
    operations, an ADD or MUL as one): from its measured instruction mix."""
    mix = measured("fp64_mix", (name,) + tuple(shape))
    if not mix:
        return {"issue_ceiling_frac": None, "frac_of_issue_ceiling": None, "fp64_instruction_mix": None}
    add, mul, fma, trans = mix
    ops, ins = add + mul + 2 * fma + trans, add + mul + fma + trans
    ceil = ops / (2.0 * ins)
    return {"issue_ceiling_frac": ceil,
            "frac_of_issue_ceiling": None if pct_hw is None else pct_hw / 100.0 / ceil,
            "fp64_instruction_mix": {"add": add, "mul": mul, "fma": fma, "trans": trans,
                                     "unit": "FP64 VALU lane-instructions per update"}}


def fma_probe(T):
    """Attainable FP64 rate measured now with the library's FMA probe (8
    independent chains per lane, 4 wavefronts per SIMD)."""
    tf, ms = T.fp64_fma_probe(8, 256 * 4 * 4 * 64 // 256, 256, 1 << 16)
    return {"tflops": tf, "ms": ms, "frac_of_spec": tf / FP64_VECTOR_PEAK_TFLOPS,
            "config": "8 FMA chains per lane, 4 wavefronts per SIMD, 65,536 iterations"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--graph", type=int, default=100, help="steps per captured HIP graph (0 = plain launches)")
    ap.add_argument("--tile", type=int, default=0, help="r* nodes per segment (0 = library default)")
    ap.add_argument("--shape", default="", help="headline launch shape 'sweep,segcols,block[,fuse]' (default: autotuned)")
    ap.add_argument("--headline-only", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-instances", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the r*-slab decomposition across GPUs is described, not built)", file=sys.stderr)
        sys.exit(2)
    torch = _torch()
    from paper_1006_0663_amd import inputs, teuk as T
    T.lib()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    from paper_1006_0663_amd import opcount
    w = inputs.C2
    log("bench: generating %s inputs" % w.name)
    fields = inputs.initial_fields(w)
    log("bench: timing %s, %d warmup + %d steps" % (w.name, args.warmup, args.steps))
    fixed = tuple(int(x) for x in args.shape.split(",")) if args.shape else None
    ms, wall, finite, shape, replays, gsteps = time_single(T, w, fields, args.steps, args.warmup, args.graph,
                                                           args.tile, torch, stream, log, fixed)
    pts = w.n_r * w.n_theta
    value = pts * args.steps / (ms / 1e3)
    ms_step = ms / args.steps
    bpu = opcount.bytes_per_update(1)
    ns = launch_steps(shape, args.steps)  # steps per launch
    launch_s = ms_step * ns / 1e3       # one launch advances ns steps
    achieved = bpu * pts * ns / launch_s / 1e9
    fpu = opcount.flops_per_update(1)
    traffic = traffic_bytes = None
    kib = measured("traffic", tuple(shape[:3]) + (ns,))
    if kib:
        traffic_bytes = 1024.0 * (kib[0] * MEASURED["fetch_scale"] + kib[1] * MEASURED["write_scale"])
        traffic = traffic_bytes / launch_s / 1e9
    fhw = measured("fp64_flops_hw", (w.name,) + tuple(shape))
    out = {
        "metric": "grid-point updates/sec per precision (FP64/dd/qd) + % FP64 peak; batched vs plain",
        "value": value, "unit": "grid-point updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "teukolsky-lw fp64 s=-2 m=2 a/M=0.9 4096x128 r*[-200,800] cfl=%g steps=%d"
                               % (w.cfl, w.steps),
                   "n_r": w.n_r, "n_theta": w.n_theta, "words": 1,
                   "graph_steps": graph_length(args.graph, args.steps), "graph_replays_timed": replays,
                   "timed_steps_in_graphs": gsteps,
                   "sweep": SWEEP_NAMES[shape[0]], "segcols": shape[1], "block": shape[2],
                   "steps_per_launch": ns},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "kernel": kernel_name(shape, ns, w.n_theta),
                     "algorithmic_bytes_per_update": bpu, "updates_per_launch": pts * ns,
                     "steps_per_launch": ns, "launch_us": launch_s * 1e6},
        "fp64_flops_per_update": fpu,
        "pct_fp64_peak": 100.0 * fpu * value / (FP64_VECTOR_PEAK_TFLOPS * 1e12),
        "fp64_flops_per_update_hw": fhw,
        "pct_fp64_peak_hw": None if fhw is None else 100.0 * fhw * value / (FP64_VECTOR_PEAK_TFLOPS * 1e12),
        "finite": finite,
        "wall_s_timed": wall,
        "kernel_source_digest": kernel_source_digest(),
    }
    out.update(issue_ceiling(w.name, shape, out["pct_fp64_peak_hw"]))
    if not args.headline_only:
        log("bench: FP64 FMA probe")
        out["fp64_fma_probe"] = fma_probe(T)
        per = {"fp64-4096x128": {"words": 1, "steps": args.steps, "updates_per_s": value, "ms_per_step": ms_step,
                                 "sweep": SWEEP_NAMES[shape[0]], "segcols": shape[1],
                                 "block": shape[2], "steps_per_launch": ns, "graph_replays_timed": replays,
                                 "pct_fp64_peak": out["pct_fp64_peak"],
                                 "pct_fp64_peak_hw": out["pct_fp64_peak_hw"],
                                 "issue_ceiling_frac": out["issue_ceiling_frac"],
                                 "frac_of_issue_ceiling": out["frac_of_issue_ceiling"]}}
        for wx in (inputs.C1, inputs.C3, inputs.C3_PARITY, inputs.C4, inputs.C2_DD, inputs.C2_QD):
            log("bench: timing %s (%d steps)" % (wx.name, wx.steps))
            fx = inputs.initial_fields(wx)
            msx, _, fin, shp, rpx, _ = time_single(T, wx, fx, wx.steps, min(args.warmup, wx.steps // 10),
                                                   args.graph, args.tile, torch, stream, log)
            ups = wx.n_r * wx.n_theta * wx.steps / (msx / 1e3)
            f = opcount.flops_per_update(wx.words)
            fh = measured("fp64_flops_hw", (wx.name,) + tuple(shp))
            per[wx.name] = {"words": wx.words, "steps": wx.steps, "updates_per_s": ups,
                            "ms_per_step": msx / wx.steps, "sweep": SWEEP_NAMES[shp[0]],
                            "segcols": shp[1], "block": shp[2], "steps_per_launch": launch_steps(shp, wx.steps),
                            "graph_replays_timed": rpx,
                            "fp64_flops_per_update": f,
                            "pct_fp64_peak": 100.0 * f * ups / (FP64_VECTOR_PEAK_TFLOPS * 1e12),
                            "fp64_flops_per_update_hw": fh,
                            "pct_fp64_peak_hw": None if fh is None else
                            100.0 * fh * ups / (FP64_VECTOR_PEAK_TFLOPS * 1e12),
                            "hbm_GBs_algorithmic": opcount.bytes_per_update(wx.words) * ups / 1e9,
                            "finite": fin}
            per[wx.name].update(issue_ceiling(wx.name, shp, per[wx.name]["pct_fp64_peak_hw"]))
        out["per_precision"] = per
        log("bench: host round trip of the state every step (%s)" % w.name)
        nrt = min(args.steps, 40)
        msr, _, finr, _, _, _ = time_single(T, w, fields, nrt, 2, 0, 0, torch, stream, log, fixed_shape=shape,
                                            round_trip=True)
        ups_rt = pts * nrt / (msr / 1e3)
        out["host_round_trip"] = {
            "workload": w.name, "steps": nrt, "updates_per_s": ups_rt, "ms_per_step": msr / nrt,
            "resident_over_round_trip": value / ups_rt, "finite": finr,
            "bytes_per_step_each_way": 4 * 8 * pts,
            "note": "state copied device->pinned host->device after every step (the per-step transfer "
                    "design the paper measured first, Sec. 'Implementation Details'); one step per launch, "
                    "no graphs"}
        out["batched"] = bench_batched(T, inputs, args, torch, stream, log)
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


def _field_digest(fields):
    import hashlib
    h = hashlib.sha1()
    for f in fields:
        h.update(f.tobytes())
    return h.hexdigest()


def bench_batched(T, inputs, args, torch, stream, log):
    ws = inputs.batch_workloads(n=args.batch_instances)
    steps = ws[0].steps
    log("bench: batched %d dd instances x %d steps (generating inputs)" % (len(ws), steps))
    fields = [inputs.initial_fields(w) for w in ws]
    grids = [T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl) for w in ws]
    from paper_1006_0663_amd import autotune, opcount
    b = T.TeukBatch([(w.s, w.m, w.a_over_M, g) for w, g in zip(ws, grids)], 2)
    b.set_stream(stream.cuda_stream)
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    if args.tile:
        b.set_launch(args.tile, 0)
        bshape = (-1, args.tile, 0, 1)
    else:
        bshape = autotune.tune(b, 2, [(w.n_r, w.n_theta) for w in ws], torch, stream, steps=8)[:4]
    if args.graph:
        b.use_graph(args.graph)
        b.prepare_graph()
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    pts = sum(w.n_r * w.n_theta for w in ws)
    nwarm = min(args.warmup, 50)
    with torch.cuda.stream(stream):
        b.step(nwarm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    log("bench: reading back the batched results")
    digest_b = [_field_digest([b.read_field(k, c) for c in range(4)]) for k in range(len(ws))]
    b.close()
    log("bench: plain loop over the same instances")
    hs = []
    for w, g, f in zip(ws, grids, fields):
        h = T.Teuk(w.s, w.m, w.a_over_M, g, 2)
        h.set_stream(stream.cuda_stream)
        h.set_initial(*f)
        if args.tile:
            h.set_launch(args.tile, 0)
        else:
            autotune.tune(h, 2, [(w.n_r, w.n_theta)], torch, stream, steps=8)
        if args.graph:
            h.use_graph(args.graph)
            h.prepare_graph()
        h.set_initial(*f)
        hs.append(h)
    with torch.cuda.stream(stream):
        for h in hs:
            h.step(nwarm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for h in hs:
            h.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1)
    digest_p = [_field_digest(h.fields()) for h in hs]
    for h in hs:
        h.close()
    f = opcount.flops_per_update(2)
    ub = pts * steps / (ms_b / 1e3)
    return {"instances": len(ws), "steps": steps, "points": pts, "words": 2,
            "batched_updates_per_s": ub,
            "plain_loop_updates_per_s": pts * steps / (ms_p / 1e3),
            "speedup": ms_p / ms_b,
            "batched_equals_loop": digest_b == digest_p,
            "equality_check": "SHA-1 of all four fields of every instance after warm-up + timed steps, "
                              "batched vs loop (bitwise)",
            "sweep": bshape[0], "segcols": bshape[1], "block": bshape[2], "steps_per_launch": bshape[3],
            "batched_pct_fp64_peak": 100.0 * f * ub / (FP64_VECTOR_PEAK_TFLOPS * 1e12)}


if __name__ == "__main__":
    main()
