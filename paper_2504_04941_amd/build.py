"""Builds libkr.so (host runtime, C ABI and ahead-of-time kernels) for gfx950.

The integrator's device templates (csrc/kr_device.h: one cell per lane;
csrc/kr_wide.h: one cell per wavefront; csrc/kr_group.h: one cell per lane
group), the rate-coefficient math
(csrc/kr_math.h), the cell-ordering kernels (csrc/kr_order.h), the
species advection (csrc/kr_advect.h) and the
launch-parameter struct (csrc/kr_params.h) are embedded into the library as string literals:
at network creation they are compiled together with the generated network
code by hipRTC."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkr.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _embed(src_name: str, out_name: str) -> None:
    text = open(os.path.join(CSRC, src_name)).read()
    assert ")KRSRC\"" not in text
    out = os.path.join(CSRC, out_name)
    content = 'R"KRSRC(' + text + ')KRSRC"\n'
    if not os.path.exists(out) or open(out).read() != content:
        with open(out, "w") as f:
            f.write(content)


def build(verbose: bool = False) -> str:
    _embed("kr_device.h", "kr_device_src.inc")
    _embed("kr_params.h", "kr_params_src.inc")
    _embed("kr_wide.h", "kr_wide_src.inc")
    _embed("kr_group.h", "kr_group_src.inc")
    _embed("kr_math.h", "kr_math_src.inc")
    _embed("kr_order.h", "kr_order_src.inc")
    _embed("kr_advect.h", "kr_advect_src.inc")
    _embed("kr_thermo.h", "kr_thermo_src.inc")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-result",
           "-o", LIB + ".tmp", os.path.join(CSRC, "kr_lib.hip"), "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
