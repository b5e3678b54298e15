"""Compile libpic.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpic.so")
SOURCES = [os.path.join(CSRC, f) for f in ("pic_kernels.hip", "pic_api.hip")]
HEADERS = [os.path.join(CSRC, "pic_dev.h"), os.path.join(ROOT, "include", "pic.h")]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 ops (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the kernels already issue one LDS atomic per wavefront for a run of
    # slots; the atomic optimizer would wrap it in a lane count and wait on
    # its return at once (measured: Weibel push 1501 -> 1469 us without it)
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libpic")


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


def build(force: bool = True) -> str:
    """Compile the library (always when force, else only if sources changed)."""
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + \
        SOURCES + ["-o", tmp]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL if os.environ.get("PIC_QUIET_BUILD")
                          else None)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
