"""Profiling driver: run a fixed number of steps of one workload with a fixed
launch shape, after a device-to-device copy of known size that calibrates
byte counters (run it under rocprofv3).

    python -m paper_1006_0663_amd.profile_step --workload fp64-4096x128 --steps 50 --segcols 4 --block 256
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
    a = ap.parse_args()
    w = inputs.WORKLOADS[a.workload]
    torch.cuda.set_device(0)
    src = torch.empty(COPY_MIB << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)                      # calibration: COPY_MIB MiB read + written
    torch.cuda.synchronize()
    g = T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass, w.angular_order)
    h = T.Teuk(w.s, w.m, w.a_over_M, g, w.words)
    h.set_launch(a.segcols, a.block)
    h.set_initial(*inputs.initial_fields(w))
    h.step(a.steps)
    ok = h.check_finite()
    h.close()
    print("profile_step: %s %d steps segcols=%d block=%d finite=%s copy=%d MiB"
          % (w.name, a.steps, a.segcols, a.block, ok, COPY_MIB), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
