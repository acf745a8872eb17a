"""Host logic of the autotuner and the bench driver (no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

from paper_1006_0663_amd import autotune  # noqa: E402


class _Handle:
    """Records the setter calls the autotuner makes; rejects fused shapes."""

    def __init__(self, reject_fuse=False):
        self.calls = []
        self.reject_fuse = reject_fuse

    def set_fuse(self, k):
        self.calls.append(("fuse", k))
        if self.reject_fuse and k > 1:
            from paper_1006_0663_amd.teuk import TeukError
            raise TeukError(-1, "no fused form")

    def set_launch(self, s, b):
        self.calls.append(("launch", s, b))

    def set_sweep(self, sw):
        self.calls.append(("sweep", sw))


def test_apply_orders_setters_so_every_shape_is_reachable():
    h = _Handle()
    autotune.apply(h, (2, 8, 256, 2))
    # single steps and the trivial launch first, the wanted shape last
    assert h.calls == [("fuse", 1), ("launch", 1, 0), ("sweep", 2), ("launch", 8, 256), ("fuse", 2)]
    h = _Handle()
    autotune.apply(h, (1, 4, 0))                    # three-element shapes mean one step per launch
    assert h.calls[-1] == ("fuse", 1)


def test_candidates_respect_theta_rows_and_steps():
    for words in (1, 2, 4):
        for nth in (32, 64, 128, 256):
            for sweep, seg, block, fuse in autotune.candidates(words, nth):
                assert block == 0 or block >= nth
                assert fuse in (1, 2, 4) and seg >= 1
                assert words == 1 or sweep != autotune.WIDE2
                assert fuse == 1 or words in (1, 2)


def test_cache_key_is_order_independent():
    a = autotune.key("dev", 2, [(1024, 64), (256, 32)])
    b = autotune.key("dev", 2, [(256, 32), (1024, 64)])
    assert a == b == "dev|w2|256x32;1024x64"


def test_stale_cache_entries_are_ignored(tmp_path, monkeypatch):
    """Entries written by an older tuner (four fields, no steps per launch)
    are not applied; a five-field entry is, without timing anything."""
    path = tmp_path / "cache.json"
    monkeypatch.setenv("TEUK_TUNE_CACHE", str(path))

    class _Torch:
        class cuda:
            @staticmethod
            def get_device_name(i):
                return "dev"

    k = autotune.key("dev", 1, [(64, 32)])
    path.write_text(json.dumps({k: [2, 8, 256, 2, 12.5]}))
    h = _Handle()
    best = autotune.tune(h, 1, [(64, 32)], _Torch, None)
    assert best == (2, 8, 256, 2, 12.5)
    assert h.calls[-1] == ("fuse", 2)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_counter_tables_follow_the_kernel_sources(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    shape = next(iter(bench.MEASURED["traffic"]))
    monkeypatch.setitem(bench.MEASURED, "source", bench.kernel_source_digest())
    assert bench.measured("traffic", shape) == bench.MEASURED["traffic"][shape]
    monkeypatch.setitem(bench.MEASURED, "source", "not-these-sources")
    assert bench.measured("traffic", shape) is None
    for key in bench.MEASURED["fp64_flops_hw"]:
        assert len(key) == 5 and key[4] in (1, 2, 4)


def test_graph_length_covers_whole_graphs_only():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.graph_length(100, 20) == 0           # shorter than one graph: plain launches
    assert bench.graph_length(100, 100) == 100
    assert bench.graph_length(100, 10000) == 100
    assert bench.graph_length(0, 20000) == 0


def test_issue_ceiling_from_the_instruction_mix(monkeypatch):
    """All-FMA code can reach the whole FP64 peak; add-only code half of it."""
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setitem(bench.MEASURED, "source", bench.kernel_source_digest())
    table = {("x", 1, 4, 256, 1): (80.0, 10.0, 10.0, 0.0), ("fma", 1, 4, 256, 1): (0.0, 0.0, 5.0, 0.0),
             ("add", 1, 4, 256, 1): (7.0, 0.0, 0.0, 0.0)}
    monkeypatch.setitem(bench.MEASURED, "fp64_mix", table)
    r = bench.issue_ceiling("x", (1, 4, 256, 1), 30.0)
    assert abs(r["issue_ceiling_frac"] - 110.0 / 200.0) < 1e-12
    assert abs(r["frac_of_issue_ceiling"] - 0.30 / 0.55) < 1e-12
    assert bench.issue_ceiling("fma", (1, 4, 256, 1), None)["issue_ceiling_frac"] == 1.0
    assert bench.issue_ceiling("add", (1, 4, 256, 1), None)["issue_ceiling_frac"] == 0.5
    assert bench.issue_ceiling("y", (1, 4, 256, 1), 10.0)["issue_ceiling_frac"] is None


def test_slab_shapes_in_the_bench_line():
    """A slab launch runs the whole timed call (up to the library's 4096 steps
    per launch); fused shapes their own step count.  The roofline names the
    kernel instance: columns per lane = segcols / (block / n_theta)."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.launch_steps((3, 16, 1024, 1), 20) == 20
    assert bench.launch_steps((3, 16, 1024, 1), 10000) == 4096
    assert bench.launch_steps((2, 16, 512, 4), 20) == 4
    assert bench.kernel_name((3, 16, 1024, 1), 20, 128) == "lw_slab_kernel<1024,2> (persistent, 20 steps per launch)"
    assert bench.kernel_name((2, 16, 512, 4), 4, 128) == "lw_wide_kernel<double,run 2> (4 steps per launch)"
    assert bench.SWEEP_NAMES[autotune.SLAB] == "slab"


def test_slab_candidates_take_one_step_setting():
    for words in (1, 2, 4):
        slab = [c for c in autotune.candidates(words, 64) if c[0] == autotune.SLAB]
        assert slab and all(c[3] == 1 for c in slab)
