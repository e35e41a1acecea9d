"""The host mesh code (checks, half-edge matching, scaled normals, reverse
Cuthill-McKee order) built for the CPU with AddressSanitizer and
UndefinedBehaviorSanitizer and run on valid meshes (jittered and relabelled
triangulations up to 180 000 triangles, two disconnected components) and on
every rejected form (bad vertex index, clockwise, degenerate, non-manifold and
same-direction neighbours, invalid mesh descriptions).  No GPU involved."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_2601_04826_amd", "csrc", "sme_mesh.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_mesh_code_under_sanitizers(tmp_path):
    exe = tmp_path / "mesh_harness"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wextra", "-Werror",
           os.path.join(HERE, "mesh_harness.cpp"), SRC, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "ALL OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    for case in ("one_square", "jittered_300", "two_components", "negative_vertex", "non_manifold",
                 "same_direction", "check_mesh"):
        assert f"OK {case}" in r.stdout
