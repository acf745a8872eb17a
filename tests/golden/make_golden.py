"""Write full-size oracle reference data for the GPU parity tests.

For each workload: build the oracle's 450-bit tables, evolve the seeded
initial data with the oracle's fixed-point engine for the workload's full
step count, and store (numpy .npz, no pickles)
  * the exact largest modulus over all components and points (4 words),
  * every component at a seeded sample of grid points plus the points of
    largest |Phi| and |Pi|, each rounded to 4 float64 words (~212 bits),
  * the workload description.
Only oracle/ and the input generator are called.  Usage:
    python tests/golden/make_golden.py [name ...] [--threads N]
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import engine, problem          # noqa: E402
from paper_1006_0663_amd import inputs      # noqa: E402

NSAMPLE = 1500


def _int_words(X, words=4):
    return inputs._int_to_words(X, engine.FRAC, words)


def workloads():
    out = {w.name: w for w in (inputs.C1, inputs.C3_PARITY, inputs.C4, inputs.C2, inputs.S0_KERR)}
    batch = inputs.batch_workloads()
    small = sorted(batch, key=lambda w: w.n_r * w.n_theta)[:2]
    for w in small:
        out[w.name] = w
    return out


def make(w, threads):
    t0 = time.time()
    p = problem.Problem(w.s, w.m, w.a_over_M, w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass,
                        w.angular_order)
    fields = inputs.initial_fields(w)
    tab = problem.build_tables(p, processes=threads)
    t1 = time.time()
    out = engine.run_problem(p, fields, w.steps, processes=threads, tables=tab)
    t2 = time.time()
    n = w.n_r * w.n_theta
    comps = [out[c * n:(c + 1) * n] for c in range(4)]
    maxabs = max(abs(v) for c in comps for v in c)
    rng = np.random.default_rng(1234)
    pts = set(int(x) for x in rng.choice(n, size=min(NSAMPLE, n), replace=False))
    for pair in ((0, 1), (2, 3)):
        mag = [comps[pair[0]][q] ** 2 + comps[pair[1]][q] ** 2 for q in range(n)]
        pts.add(int(np.argmax(np.array([float(v) for v in mag]))))
    pts = sorted(pts)
    vals = np.array([[_int_words(comps[c][q]) for c in range(4)] for q in pts])   # [npts][4][4]
    np.savez_compressed(os.path.join(HERE, "%s.npz" % w.name),
                        points=np.array(pts, dtype=np.int64), values=vals,
                        maxabs=np.array(_int_words(maxabs)),
                        workload=np.array(json.dumps(dataclasses.asdict(w))),
                        oracle_seconds=np.array([t1 - t0, t2 - t1]))
    print("%s: tables %.0fs, %d steps %.0fs, max %.3e" % (w.name, t1 - t0, w.steps, t2 - t1,
                                                          maxabs / 2.0 ** engine.FRAC), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    a = ap.parse_args()
    ws = workloads()
    for name in (a.names or list(ws)):
        make(ws[name], a.threads)


if __name__ == "__main__":
    main()
