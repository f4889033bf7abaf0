"""Build the HIP library (libarna.so) for gfx950 in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "arna.hip")
# k_run is compiled on its own, with machine-level loop-invariant code motion
# off: hoisting constants out of its iteration loop holds them in registers
# across the loop and spills
SRC_RUN = os.path.join(PKG, "csrc", "arna_run.hip")
DEPS = [SRC, SRC_RUN, os.path.join(PKG, "csrc", "arna_device.hpp"),
        os.path.join(PKG, "csrc", "arna_kernels.hpp"), os.path.join(PKG, "csrc", "arna_adjoint.hpp"),
        os.path.join(PKG, "csrc", "arna_stream.hpp"), os.path.join(PKG, "csrc", "arna_master.hpp"),
        os.path.join(ROOT, "include", "arna.h")]
LIB = os.path.join(PKG, "libarna.so")
ARCH = "gfx950"
# packed FP32 instructions stay off (they are not used by this code)
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
RUN_FLAGS = ["-mllvm", "-disable-machine-licm"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def commands(out: str, objdir: str) -> list:
    """hipcc command lines: one object per translation unit, then the link."""
    inc = ["-I", os.path.join(ROOT, "include")]
    o_main = os.path.join(objdir, "arna.o")
    o_run = os.path.join(objdir, "arna_run.o")
    arch = f"--offload-arch={ARCH}"
    return [[hipcc(), arch, *FLAGS, *inc, "-c", "-o", o_main, SRC],
            [hipcc(), arch, *FLAGS, *RUN_FLAGS, *inc, "-c", "-o", o_run, SRC_RUN],
            [hipcc(), arch, "-fPIC", "-shared", "-o", out, o_main, o_run]]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory() as objdir:
        cmds = commands(tmp, objdir)
        # the two translation units compile in parallel
        procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
                 for c in cmds[:2]]
        outs = [p.communicate() for p in procs]
        for p, (o, e) in zip(procs, outs):
            if p.returncode != 0:
                raise RuntimeError("hipcc failed:\n" + o + e)
            if verbose:
                print(e)
        res = subprocess.run(cmds[2], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
