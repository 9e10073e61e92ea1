"""Build the gfx950 HIP library liblagrangeflux.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SO = os.path.join(PKG, "liblagrangeflux.so")
SOURCES = ["lf_api.hip", "lf_forward.hip", "lf_fused.hip", "lf_adjoint.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no implicit contraction: every fused multiply-add in the kernels is
    # written explicitly, so x- and y-faces round identically
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(out: str = SO, extra_flags=()) -> str:
    """Compile every source to an object in parallel, then link the shared
    library (the kernels of one file never call into another)."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="lf_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]

        def compile_one(src_obj):
            src, obj = src_obj
            subprocess.run([hipcc(), *compile_flags, *extra_flags, "-I", os.path.join(ROOT, "include"),
                            "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj], check=True)

        with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as pool:
            list(pool.map(compile_one, zip(SOURCES, objs)))
        tmp = out + ".tmp"
        subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *extra_flags, "-o", tmp, *objs],
                       check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))
