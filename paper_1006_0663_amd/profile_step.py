"""Profiling driver: run a fixed number of steps of one workload with a fixed
launch shape (or the autotuner's, from its cache when present), after a
device-to-device copy of known size that calibrates byte counters (run it
under rocprofv3).

    python -m paper_1006_0663_amd.profile_step --workload fp64-4096x128 --steps 50 --sweep 1 --segcols 16 --block 512
    python -m paper_1006_0663_amd.profile_step --workload fp64-4096x128 --steps 50 --tuned
"""
import argparse
import sys

import torch

from paper_1006_0663_amd import inputs, teuk as T

COPY_MIB = 256


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="fp64-4096x128", choices=sorted(inputs.WORKLOADS))
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--segcols", type=int, default=4)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--sweep", type=int, default=-1,
                    help="0 segment, 1 wide, 2 wide with runs of two, 3 slab (persistent; --steps in one launch), "
                         "-1 default")
    ap.add_argument("--fuse", type=int, default=1, help="steps per launch (1, 2 or 4)")
    ap.add_argument("--tuned", action="store_true", help="use the autotuner's shape (cached if tuned before)")
    ap.add_argument("--time", type=int, default=0, metavar="REPS",
                    help="also time REPS runs of --steps graph-replayed steps (HIP events) and print us/step")
    ap.add_argument("--dd-coef", choices=("0", "3", "4"), default=None,
                    help="double-double coefficient source (sets TEUK_DD_COEF): 0 stored planes, "
                         "3 planes requested one phase ahead, 4 rebuilt per point")
    a = ap.parse_args()
    if a.dd_coef is not None:
        import os
        os.environ["TEUK_DD_COEF"] = a.dd_coef          # read when the handle is created
    w = inputs.WORKLOADS[a.workload]
    torch.cuda.set_device(0)
    src = torch.empty(COPY_MIB << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)                      # calibration: COPY_MIB MiB read + written
    torch.cuda.synchronize()
    g = T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass, w.angular_order)
    h = T.Teuk(w.s, w.m, w.a_over_M, g, w.words)
    h.set_initial(*inputs.initial_fields(w))
    if a.tuned:
        from paper_1006_0663_amd import autotune
        stream = torch.cuda.current_stream()
        h.set_stream(stream.cuda_stream)
        a.sweep, a.segcols, a.block, a.fuse, _ = autotune.tune(h, w.words, [(w.n_r, w.n_theta)], torch, stream)
        h.set_initial(*inputs.initial_fields(w))
    else:
        h.set_sweep(a.sweep)
        h.set_launch(a.segcols, a.block)
        h.set_fuse(a.fuse)
    h.step(a.steps)
    timing = ""
    if a.time:
        stream = torch.cuda.Stream()
        h.set_stream(stream.cuda_stream)
        h.use_graph(min(100, a.steps))
        h.prepare_graph()
        with torch.cuda.stream(stream):
            h.step(a.steps)                     # warm-up (clocks, caches)
            ts = []
            for _ in range(a.time):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                h.step(a.steps)
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e3 / a.steps)
        timing = " us_per_step_min=%.3f all=%s" % (min(ts), ",".join("%.3f" % t for t in ts))
    ok = h.check_finite()
    h.close()
    print("profile_step: %s %d steps sweep=%d segcols=%d block=%d fuse=%d finite=%s copy=%d MiB%s%s"
          % (w.name, a.steps, a.sweep, a.segcols, a.block, a.fuse, ok, COPY_MIB,
             "" if a.dd_coef is None else " dd_coef=" + a.dd_coef, timing), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
