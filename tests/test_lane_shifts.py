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
import re

import pytest


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
def test_no_lane_shift_in_divergent_code(src, kernel_asm):
    asm = kernel_asm[src]
    assert "_dpp" in asm  # the kernels do use lane shifts
    assert _shifts_in_divergent_code(asm) == {}
