"""The band-height chooser of the structured step (host logic, built for the
CPU with hipcc's host pass and run without a GPU): the choices its comment
documents for the grids it was measured on, and the properties of its two
cost models."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_04826_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HARNESS = r"""
#include "sme_host.h"
#include <cstdio>
#include <cstdlib>
namespace sme { int step_2d_waves_per_simd(int) { return 1; } }
int main(int argc, char **argv)
{
    for (int k = 1; k + 3 < argc; k += 4)
        std::printf("%d\n", sme::host::pick_rows_for(atoi(argv[k]), atoll(argv[k + 1]), atoll(argv[k + 2]),
                                                     atoi(argv[k + 3])));
    return 0;
}
"""


@pytest.fixture(scope="module")
def pick(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("rows")
    src, exe = d / "h.cpp", d / "h"
    src.write_text(HARNESS)
    r = subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]

    def run(cases):
        args = [str(v) for c in cases for v in c]
        out = subprocess.run([str(exe)] + args, capture_output=True, text=True, check=True).stdout.split()
        return [int(x) for x in out]

    return run


def test_documented_choices(pick):
    # (waves per SIMD, nx, ny, compute units) -> rows
    cases = {(2, 1024, 1024, 256): 9,    # one generation: 17 strips x 114 bands = 1938 <= 2048 slots
             (2, 2048, 2048, 256): 35,   # one generation of 2006 waves
             (2, 3072, 3072, 256): 38,   # in step: 1.98 generations
             (2, 4096, 4096, 256): 16,   # drift model
             (3, 4096, 4096, 256): 11,
             (2, 6144, 6144, 256): 24,
             (6, 8192, 8192, 256): 16,
             (1, 2048, 2048, 256): 35}   # one wave per SIMD: always in step
    assert pick(list(cases)) == list(cases.values())


def test_single_generation_takes_the_shortest_band_that_fits(pick):
    for ps, n in [(2, 1024), (3, 1024), (6, 1024), (2, 700), (1, 1500)]:
        slots, nsx = 256 * 4 * ps, (n + 61) // 62
        r, = pick([(ps, n, n, 256)])
        fits = lambda rows: nsx * -(-n // rows) <= slots
        if fits(64):
            assert fits(r) and (r == 2 or not fits(r - 1)), (ps, n, r)


def test_band_is_at_least_two_and_at_most_64_rows(pick):
    cases = [(ps, n, n, cu) for ps in (1, 2, 4, 8) for n in (1, 62, 63, 500, 5000, 20000) for cu in (1, 256)]
    for r in pick(cases):
        assert 2 <= r <= 64
