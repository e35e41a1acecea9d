"""Host logic of bench.py (CPU): algorithmic bytes per cell, the committed
counter figures (HBM traffic, executed FP64 flops) that are reported only while
the sources of their workload still hash to the value they were taken on, and
the clock warm-up before the timed steps."""
import json
import os
import time

import bench


def test_bytes_per_cell():
    # read every field and the bathymetry once, write every field once
    assert bench.bytes_per_cell("2d", 2) == (7 * 2 + 1) * 8 == 120
    assert bench.bytes_per_cell("2d", 8) == (19 * 2 + 1) * 8 == 312
    assert bench.bytes_per_cell("1d", 1) == (3 * 2 + 1) * 8 == 56
    # triangles add 3 int32 neighbours and 3 x (n_x, n_y, |e|/|V|) FP64
    assert bench.bytes_per_cell("tri", 3) == (9 * 2 + 1) * 8 + 12 + 48 + 8 == 220


def test_counter_figures_follow_the_source_hash(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2601_04826_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("// kernel v1\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.source_hash()
    (tmp_path / "profiles" / "traffic_w.json").write_text(json.dumps({"source_hash": h, "bytes_per_launch": 123.0}))
    (tmp_path / "profiles" / "flops_w.json").write_text(json.dumps({"source_hash": h, "fp64_flops_per_launch": 4.5e9}))
    assert bench.load_traffic("w", 100.0) == 123.0
    assert bench.load_flops("w") == 4.5e9
    assert bench.load_traffic("other", 100.0) is None and bench.load_flops("other") is None
    # any change to a kernel source invalidates both
    (csrc / "k.hip").write_text("// kernel v2\n")
    assert bench.source_hash() != h
    assert bench.load_traffic("w", 100.0) is None
    assert bench.load_flops("w") is None


def test_workload_hash_covers_its_own_sources_and_every_header(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2601_04826_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("k_step_2d.hip", "k_vam.hip", "k_misc.hip", "sme_lib.cpp", "common.h"):
        (csrc / f).write_text(f"// {f} v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    wl = "struct_2d_1024_l2"
    h = bench.source_hash(wl)
    (csrc / "k_vam.hip").write_text("// another kernel, changed\n")
    assert bench.source_hash(wl) == h
    assert bench.source_hash() != h  # the whole-library hash sees it
    for f in ("k_step_2d.hip", "sme_lib.cpp", "k_misc.hip", "common.h"):
        (csrc / f).write_text("// changed\n")
        assert bench.source_hash(wl) != h, f
        h = bench.source_hash(wl)
    assert set(bench.WORKLOAD_SOURCES) == set(bench.WORKLOADS)
    real = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2601_04826_amd", "csrc")
    for files in bench.WORKLOAD_SOURCES.values():
        for f in files:
            assert os.path.exists(os.path.join(real, f)), f


def test_clock_warmup_runs_until_its_time_is_spent():
    calls = []

    class FakeCuda:
        @staticmethod
        def synchronize():
            calls.append("sync")

    class FakeTorch:
        cuda = FakeCuda

    def chunk():
        calls.append("chunk")
        time.sleep(0.01)

    el = bench.warm_clocks(FakeTorch, chunk, 0.05)
    assert el >= 0.05
    n = calls.count("chunk")
    assert 5 <= n <= 20 and calls.count("sync") == n
    calls.clear()
    assert bench.warm_clocks(FakeTorch, chunk, 0.0) >= 0.0 and calls.count("chunk") == 1  # always one chunk


def test_committed_workloads_are_known():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for f in os.listdir(os.path.join(root, "profiles")):
        if f.endswith(".json"):
            wl = f.split("_", 1)[1][:-5]
            assert wl in bench.WORKLOADS, f


def test_vam_bytes_per_cell():
    import bench

    # one block (two cells): no reduction level, only the top equation of each solve
    two = bench.vam_bytes_per_cell(2)
    assert two == (88 * 2 + 256 * 2 + 80 * 2 + 80 * 2 + 96 * 2 + 8 * (76 + 24)) / 2
    # a level of n equations: 104 n words in the first solve, 32 n in the
    # second, 24 n per back substitution; the levels sum to about 2 nb = nx
    big = bench.vam_bytes_per_cell(1 << 20)
    per_cell = 88 + 256 + 80 + 80 + 96 + 8 * (104 + 32 + 2 * 24)
    assert abs(big - per_cell) < 0.01 * per_cell
