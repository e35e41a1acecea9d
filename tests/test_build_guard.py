"""Register-spill guard of the build (CPU only: hipcc cross-compiles gfx950).

The guard reads the compiler's kernel-resource-usage remarks and fails the
build when a kernel spills more SGPRs than the level-8 structured step does
with machine loop-invariant code motion disabled, spills VGPRs or uses
scratch.  These tests check the remark parser on a fixed text, the limits, and
that the guard trips on the configuration it exists for (the structured step
compiled with loop-invariant code motion enabled).
"""
import os
import subprocess

import pytest

from paper_2601_04826_amd import build

REMARKS = """\
k.hip:1:1: remark: Function Name: _Z3fooPd [-Rpass-analysis=kernel-resource-usage]
k.hip:1:1: remark:     TotalSGPRs: 106 [-Rpass-analysis=kernel-resource-usage]
k.hip:1:1: remark:     VGPRs: 168 [-Rpass-analysis=kernel-resource-usage]
k.hip:1:1: remark:     ScratchSize [bytes/lane]: 24 [-Rpass-analysis=kernel-resource-usage]
k.hip:1:1: remark:     SGPRs Spill: 37 [-Rpass-analysis=kernel-resource-usage]
k.hip:1:1: remark:     VGPRs Spill: 6 [-Rpass-analysis=kernel-resource-usage]
k.hip:2:1: remark: Function Name: _Z3barPd [-Rpass-analysis=kernel-resource-usage]
k.hip:2:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:2:1: remark:     SGPRs Spill: 255 [-Rpass-analysis=kernel-resource-usage]
k.hip:2:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
"""


def test_parser_reads_every_kernel():
    assert build.resource_usage(REMARKS) == [("_Z3fooPd", 37, 6, 24), ("_Z3barPd", 255, 0, 0)]


def test_limits():
    build.check_spills("k.hip", [("_Z3barPd", 255, 0, 0)])  # at the limit: passes
    for bad in [("a", 256, 0, 0), ("b", 0, 1, 0), ("c", 0, 0, 8)]:
        with pytest.raises(RuntimeError, match="spill guard"):
            build.check_spills("k.hip", [bad])


def test_build_flags_keep_licm_off():
    assert "-disable-machine-licm" in build.FLAGS


@pytest.mark.skipif(not os.path.exists(build.HIPCC), reason="hipcc not installed")
def test_guard_trips_on_structured_step_with_licm(tmp_path):
    flags = [f for f in build.FLAGS if f not in ("-mllvm", "-disable-machine-licm")]
    # keep the other -mllvm options paired (none today besides the LICM switch)
    assert "-mllvm" not in flags
    cmd = [build.HIPCC, build.REMARKS] + flags + ["--cuda-device-only", "-c",
                                                 os.path.join(build.CSRC, "k_step_2d.hip"), "-o", str(tmp_path / "k.o")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    usage = build.resource_usage(r.stdout + r.stderr)
    level8 = [u for u in usage if "k_step_2dILi8E" in u[0]]
    assert level8 and max(u[1] for u in level8) > build.MAX_SGPR_SPILL
    with pytest.raises(RuntimeError, match="spill guard"):
        build.check_spills("k_step_2d.hip", usage)
