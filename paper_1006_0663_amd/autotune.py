"""Autotuner for the step kernel's launch shape.

Times a short run of every candidate (segment length S, block size) on the
actual instance or batch with HIP events on the handle's stream, keeps the
fastest, and caches the choice in a JSON file keyed by device, precision and
grid shape (``TEUK_TUNE_CACHE``, default tune_cache.json next to this file).  The
launch shape does not change results (tested bitwise), only speed.
"""
import json
import os

SEGCOLS = (1, 2, 3, 4, 6, 8, 12, 16)
BLOCKS = (0, 128, 256)


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


def candidates(max_nth):
    out = []
    for b in BLOCKS:
        if b and b < max_nth:
            continue
        for s in SEGCOLS:
            out.append((s, b))
    return out


def tune(handle, words, shapes, torch, stream, steps=20, reps=2, use_cache=True, log=None):
    """Pick the fastest (segcols, block) for `handle` (Teuk or TeukBatch, already
    holding valid fields and set to `stream`).  Returns (segcols, block, us_per_step)."""
    dev = torch.cuda.get_device_name(0)
    k = key(dev, words, shapes)
    db = _load() if use_cache else {}
    if k in db:
        s, b, t = db[k]
        handle.set_launch(s, b)
        return s, b, t
    best = None
    max_nth = max(n for _, n in shapes)
    for s, b in candidates(max_nth):
        handle.set_launch(s, b)
        with torch.cuda.stream(stream):
            handle.step(2)
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
            log("tune %s: segcols=%d block=%d %.2f us/step" % (k, s, b, t))
        if best is None or t < best[2]:
            best = (s, b, t)
    handle.set_launch(best[0], best[1])
    if use_cache:
        db = _load()
        db[k] = list(best)
        _store(db)
    return best
