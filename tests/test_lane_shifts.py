"""Build-time guard on the device code: every DPP lane shift in the HIP
kernels must execute with the whole wave active.

The stage and adjoint kernels exchange neighbour values with whole-wave
DPP shifts.  Inside control flow that narrows the EXEC mask, a shift
reads inactive lanes as zero, which silently corrupts the neighbour
value.  The compiler may create such control flow by itself (turning a
select into a branch and moving a shift into one arm), so this test
compiles the kernels for gfx950 to assembly and checks that no DPP
instruction lies between an EXEC-narrowing instruction and the
restoring one."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_08710_amd", "csrc")


def _assembly(src, tmp_path):
    from paper_1607_08710_amd import _build
    out = str(tmp_path / (src + ".s"))
    flags = [f for f in _build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [_build.hipcc(), *flags, "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-o", out, os.path.join(CSRC, src)]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read()


def _shifts_in_divergent_code(asm):
    found = {}
    for m in re.finditer(r"^(_ZN2lf\w+):", asm, re.M):
        start = m.end()
        end = asm.index(".Lfunc_end", start)
        narrowed, count = False, 0
        for line in asm[start:end].split("\n"):
            t = line.strip()
            if re.match(r"s_\w+_saveexec_b64", t) or re.match(r"s_(and|andn2|mov)_b64 exec,", t):
                narrowed = True
            if re.match(r"s_or_b64 exec, exec", t):
                narrowed = False
            if narrowed and "_dpp" in t:
                count += 1
        if count:
            found[m.group(1)] = count
    return found


@pytest.mark.parametrize("src", ["lf_forward.hip", "lf_fused.hip", "lf_adjoint.hip"])
def test_no_lane_shift_in_divergent_code(src, tmp_path):
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not installed")
    asm = _assembly(src, tmp_path)
    assert "_dpp" in asm  # the kernels do use lane shifts
    assert _shifts_in_divergent_code(asm) == {}
