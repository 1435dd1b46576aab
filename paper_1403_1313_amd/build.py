"""Builds libpms.so (the C-ABI library with its gfx950 kernels) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpms.so")
SOURCES = [os.path.join(CSRC, "pms_kernels.hip"), os.path.join(CSRC, "pms_group.hip"),
           os.path.join(CSRC, "pms_nbhd.hip"), os.path.join(CSRC, "pms_probe.hip"),
           os.path.join(CSRC, "pms_noalloc.hip"), os.path.join(CSRC, "pms_api.hip")]
ARCH = os.environ.get("PMS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-result",
    # keep the compiler from forming packed fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# roctx ranges around the entry points (markers for a profiler's trace)
LIBS = [f"-L{ROCM}/lib", f"-Wl,-rpath,{ROCM}/lib", "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; install ROCm or set HIPCC")


def build_id() -> str:
    """Hash of the library's sources and headers (keys the autotune cache)."""
    import hashlib
    h = hashlib.sha256()
    for path in sorted(SOURCES + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
                       + [os.path.join(INCLUDE, "pms.h")]):
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()[:12]


def build(out: str = LIB, extra=(), verbose: bool = False) -> str:
    tmp = out + ".tmp"
    cmd = [hipcc(), *FLAGS, f'-DPMS_BUILD_ID="{build_id()}"', *extra, *SOURCES, *LIBS, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    if verbose:
        noise = "is not a recognized feature for this target"
        for line in (res.stdout + res.stderr).splitlines():
            if noise not in line:
                print(line)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
