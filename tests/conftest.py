import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liblfo.so")):
        oracle.build()
    return oracle


def params_from(cfg, **over):
    import oracle
    kw = dict(nx=cfg["nx"], ny=cfg["ny"], dx=cfg["dx"], dy=cfg["dy"], gamma=cfg["gamma"],
              cfl=cfg["cfl"], beta=cfg["beta"], bc_x=cfg["bc_x"], bc_y=cfg["bc_y"],
              ns=cfg.get("ns", 0), recon=cfg.get("recon", 0))
    kw.update(over)
    return oracle.Params(**kw)


def read_golden(name):
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def kernel_asm(tmp_path_factory):
    """gfx950 assembly of each HIP source of the library, compiled once per
    session (in parallel) for the tests that inspect the generated code."""
    import subprocess
    from concurrent.futures import ThreadPoolExecutor
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not installed")
    from paper_1607_08710_amd import _build
    tmp = tmp_path_factory.mktemp("asm")
    flags = [f for f in _build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    srcs = ["lf_forward.hip", "lf_fused.hip", "lf_adjoint.hip"]

    def one(src):
        out = str(tmp / (src + ".s"))
        subprocess.run([_build.hipcc(), *flags, "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
                        "-I", _build.CSRC, "-o", out, os.path.join(_build.CSRC, src)],
                       check=True, capture_output=True)
        with open(out) as fh:
            return src, fh.read()

    with ThreadPoolExecutor(max_workers=len(srcs)) as pool:
        return dict(pool.map(one, srcs))
