"""The single-pass step kernel is bound by VALU issue, and bench.py prices
it with the number of VALU instructions its main loop takes per row (a
predictor row and a corrector row with the CFL reduction, per lane = per
cell) in the gfx950 assembly.  The loop runs three rows per trip; this
test recounts the trip from a fresh compile, so the figure the benchmark
reports cannot drift from the kernel."""
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _main_loop_valu(asm, symbol):
    start = asm.index(symbol + ":")
    end = asm.index(".Lfunc_end", start)
    lines = [l.strip() for l in asm[start:end].split("\n")]
    labels = {}
    for i, l in enumerate(lines):
        m = re.match(r"^(\.LBB\S+):", l)
        if m:
            labels[m.group(1)] = i
    loops = []
    for i, l in enumerate(lines):
        m = re.search(r"s_c?branch\w*\s+(\.LBB\S+)", l)
        if m and m.group(1) in labels and labels[m.group(1)] < i:
            loops.append((labels[m.group(1)], i))
    # The main loop stores the new state.  It is rotated: one back edge
    # skips the CFL reduction block (lf_step), the other runs through it
    # (lf_advance, the timed path); the iteration counted is the latter,
    # the longest loop that stores.
    body = [lines[a:b + 1] for a, b in loops if any(x.startswith("global_store") for x in lines[a:b + 1])]
    assert body, loops
    body = max(body, key=len)
    assert any(x.startswith("v_rsq") for x in body)  # the reduction's sound speed is in it
    # rows per trip: each row stores the four fields of U^{n+1} and of the
    # optional U*
    stores = sum(1 for x in body if x.startswith("global_store"))
    assert stores % 8 == 0, stores
    return sum(1 for x in body if x.startswith("v_")) / (stores // 8)


def test_single_pass_valu_count(kernel_asm):
    sys.path.insert(0, ROOT)
    import bench
    asm = kernel_asm["lf_fused.hip"]
    got = {8: _main_loop_valu(asm, "_ZN2lf17fused_step_kernelIdLi0ELi0ELi0ELb0EEEvNS_9FusedArgsIT_EE"),
           4: _main_loop_valu(asm, "_ZN2lf17fused_step_kernelIfLi0ELi0ELi0ELb0EEEvNS_9FusedArgsIT_EE")}
    assert got == bench.VALU_OPS_PER_CELL, got


def _registers(asm):
    """Kernel name -> (VGPRs, spilled VGPRs, spilled SGPRs), from the code
    object metadata of the assembly."""
    out = {}
    for blk in asm.split("  - .agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)
        out[name] = tuple(int(re.search(r"\.%s:\s+(\d+)" % k, blk).group(1))
                          for k in ("vgpr_count", "vgpr_spill_count", "sgpr_spill_count"))
    return out


def test_kernel_registers(kernel_asm):
    """No kernel spills VGPRs to scratch memory, except the FP64 strip step
    (ghost rows) with four mass fractions under transmissive x (two
    registers).  (SGPR spills go
    to VGPR lanes, not to memory, and are not counted.)  The FP32
    single-pass step of the benchmark fits five waves per SIMD (at most 96
    VGPRs), the FP64 one three (at most 168), also as a strip step."""
    regs = {}
    for src in ("lf_forward.hip", "lf_fused.hip", "lf_adjoint.hip"):
        regs.update(_registers(kernel_asm[src]))
    assert len(regs) > 200
    spills = {k: v[1] for k, v in regs.items() if v[1]}
    assert spills == {"_ZN2lf17fused_step_kernelIdLi1ELi2ELi4ELb0EEEvNS_9FusedArgsIT_EE": 2}, spills
    assert regs["_ZN2lf17fused_step_kernelIfLi0ELi0ELi0ELb0EEEvNS_9FusedArgsIT_EE"][0] <= 96
    assert regs["_ZN2lf17fused_step_kernelIdLi0ELi0ELi0ELb0EEEvNS_9FusedArgsIT_EE"][0] <= 168
    assert regs["_ZN2lf17fused_step_kernelIdLi0ELi2ELi0ELb0EEEvNS_9FusedArgsIT_EE"][0] <= 168  # strip step
