"""Autotuner for the step kernel's launch shape.

Times a short run of every candidate (sweep, segment length, block size,
steps per launch) on the actual instance or batch with HIP events on the handle's stream, keeps
the fastest, and caches the choice in a JSON file keyed by device, precision
and grid shape (``TEUK_TUNE_CACHE``, default tune_cache.json next to this
file).  The launch shape does not change results (tested bitwise), only speed.
"""
import json
import os

SEGMENT, WIDE, WIDE2, SLAB = 0, 1, 2, 3

# (sweep, segcols, block, steps per launch) per precision (words); block 0 =
# library default.  Fused launches (2 or 4 steps) pay off on small grids,
# where one step does not fill the chip and launch overhead dominates, and on
# the 4096 x 128 FP64 grid (runs of two columns: segments of 16 with four
# steps or of 8 with two; runs of one: segments of 8, blocks of 512).  The
# persistent slab sweep (FP64, n_theta a multiple of 64, every block resident
# at once) takes a call's steps in one launch; shapes whose blocks do not all
# fit on the device are refused by the library and skipped.  Double-double
# slab shapes hold their coefficients in registers (one or two columns per
# lane); quad-double ones load them per stage (one column per lane).
CANDIDATES = {
    1: [(WIDE, s, b, 1) for b in (128, 256, 512) for s in (4, 6, 8, 12, 16, 24)]
       + [(WIDE2, s, b, 1) for b in (128, 256, 512) for s in (4, 6, 8, 10, 16, 22)]
       + [(SEGMENT, 4, 256, 1), (SEGMENT, 8, 256, 1)]
       + [(WIDE, s, b, f) for f in (2, 4) for b in (256, 512) for s in (2, 4)]
       + [(WIDE, s, 512, 2) for s in (6, 8)] + [(WIDE2, 8, 256, 2), (WIDE2, 16, 512, 2), (WIDE2, 16, 512, 4)]
       + [(SLAB, s, b, 1) for b, s in ((256, 4), (256, 8), (512, 8), (512, 16), (1024, 16), (1024, 32))],
    2: [(WIDE, s, b, 1) for b in (0, 256, 512) for s in (2, 4, 6, 8, 12, 16)]
       + [(WIDE, s, 512, 1) for s in (24, 32)]
       + [(SEGMENT, 2, 0, 1), (SEGMENT, 2, 128, 1)]
       + [(WIDE, s, b, 2) for b in (256, 512) for s in (2, 4)] + [(WIDE, s, 512, 4) for s in (4, 8)]
       + [(SLAB, s, b, 1) for b, s in ((256, 4), (256, 8), (512, 4), (512, 8))],
    4: [(WIDE, s, b, 1) for b in (128, 256) for s in (2, 4, 6, 8, 12, 16)] + [(SEGMENT, 2, 128, 1), (SEGMENT, 2, 0, 1)]
       + [(SLAB, s, b, 1) for b, s in ((256, 4), (512, 8), (1024, 16))],
}


def cache_path():
    return os.environ.get("TEUK_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                          "tune_cache.json"))


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def key(device_name, words, shapes):
    """shapes: list of (n_r, n_theta) of the instances."""
    return "%s|w%d|%s" % (device_name, words, ";".join("%dx%d" % s for s in sorted(shapes)))


def candidates(words, max_nth):
    return [c for c in CANDIDATES[words] if c[2] == 0 or c[2] >= max_nth]


def apply(handle, shape):
    """shape: (sweep, segcols, block[, steps per launch])."""
    sweep, segcols, block = shape[:3]
    fuse = shape[3] if len(shape) > 3 else 1
    handle.set_fuse(1)               # single steps: every sweep and shape accepts them
    handle.set_launch(1, 0)          # a shape every sweep accepts
    handle.set_sweep(sweep)
    handle.set_launch(segcols, block)
    handle.set_fuse(fuse)


def tune(handle, words, shapes, torch, stream, steps=20, reps=3, use_cache=True, log=None):
    """Pick the fastest (sweep, segcols, block, fuse) for `handle` (Teuk or
    TeukBatch, already holding valid fields and set to `stream`), leave the
    handle set to it and return (sweep, segcols, block, fuse, us_per_step)."""
    from paper_1006_0663_amd.teuk import TeukError
    dev = torch.cuda.get_device_name(0)
    k = key(dev, words, shapes)
    db = _load() if use_cache else {}
    if k in db and len(db[k]) == 5:
        best = tuple(db[k])
        apply(handle, best[:4])
        return best
    best = None
    max_nth = max(n for _, n in shapes)
    with torch.cuda.stream(stream):
        handle.step(10 * steps)          # bring the clocks up before the first candidate
        stream.synchronize()
    for cand in candidates(words, max_nth):
        try:
            apply(handle, cand)
        except TeukError as ex:          # shape does not fit this device or grid
            if log:
                log("tune %s: %s skipped (%s)" % (k, cand, ex))
            continue
        with torch.cuda.stream(stream):
            handle.step(4)
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                handle.step(steps)
                e1.record(stream)
                e1.synchronize()
                times.append(e0.elapsed_time(e1) * 1e3 / steps)
        t = min(times)
        if log:
            log("tune %s: sweep=%d segcols=%d block=%d fuse=%d %.2f us/step" % ((k,) + tuple(cand) + (t,)))
        if best is None or t < best[4]:
            best = tuple(cand) + (t,)
    apply(handle, best[:4])
    if use_cache:
        db = _load()
        db[k] = list(best)
        _store(db)
    return best
