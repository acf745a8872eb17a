"""The device's attainable FP64 vector rate, measured with the library's FMA
probe kernel (teuk_fp64_fma_probe): a sweep over independent FMA chains per
lane and wavefronts per SIMD (256 CUs x 4 SIMDs), printed as a table and as
one JSON line with the best rate.

    python -m paper_1006_0663_amd.peak_probe
"""
import json
import sys

from paper_1006_0663_amd import teuk as T

CUS, SIMDS = 256, 4
SPEC_TFLOPS = 78.6            # MI355X FP64 vector, published


def sweep(iters=1 << 16, chains=(1, 2, 4, 8), waves_per_simd=(1, 2, 4, 8), threads=256):
    rows = []
    for wps in waves_per_simd:
        blocks = CUS * SIMDS * wps * 64 // threads
        for ch in chains:
            tf, ms = T.fp64_fma_probe(ch, blocks, threads, iters)
            rows.append({"chains": ch, "waves_per_simd": wps, "blocks": blocks, "threads": threads,
                         "iters": iters, "tflops": tf, "ms": ms, "frac_of_spec": tf / SPEC_TFLOPS})
    return rows


def best(rows):
    return max(rows, key=lambda r: r["tflops"])


def main():
    import torch
    if not torch.cuda.is_available():
        sys.exit("peak_probe needs a GPU")
    torch.cuda.set_device(0)
    rows = sweep()
    print("| chains | waves/SIMD | TFLOP/s | of 78.6 |")
    print("|---|---|---|---|")
    for r in rows:
        print("| %d | %d | %.1f | %.3f |" % (r["chains"], r["waves_per_simd"], r["tflops"], r["frac_of_spec"]))
    print(json.dumps({"best": best(rows), "spec_tflops": SPEC_TFLOPS}), flush=True)


if __name__ == "__main__":
    main()
