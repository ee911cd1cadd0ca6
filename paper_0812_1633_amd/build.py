"""Build the HIP library ``libre_hip.so`` for gfx950 (in-tree).

hipcc compiles the kernels and the host runtime into one shared library with
a plain C ABI (``include/re.h``).  Packed FP32 instructions are disabled for
every device compilation.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libre_hip.so")
SOURCES = ["re_kernels.hip", "re_persist.hip", "re_host.cpp", "re_tune.cpp"]
ARCH = os.environ.get("RE_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def build(verbose: bool = False, defines=(), lib_path: str = LIB) -> str:
    """Compile every source (in parallel) and link libre_hip.so.

    ``defines`` adds preprocessor symbols (e.g. ``RE_PHASE_TIMERS`` for a
    build with the persistent kernel's phase timers, written to another
    ``lib_path``)."""
    tag = "_".join(defines)
    objdir = os.path.join(HERE, "_build" + ("_" + tag if tag else ""))
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc()] + FLAGS + ["-D" + d for d in defines] + ["-c", path, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        # hipcc's host pass does not know the packed-fp32 feature; harmless
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if p.returncode != 0:
            failed.append((cmd, out))
        elif verbose and out:
            print(out)
    if failed:
        msg = "\n\n".join(" ".join(c) + "\n" + o for c, o in failed)
        raise RuntimeError("HIP build failed:\n" + msg)
    tmp = lib_path + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="build libre_hip.so for gfx950")
    ap.add_argument("--phase-timers", action="store_true",
                    help="build libre_hip_timers.so instead, with the persistent kernel's phase timers")
    a = ap.parse_args()
    if a.phase_timers:
        print(build(verbose=True, defines=("RE_PHASE_TIMERS",), lib_path=os.path.join(HERE, "libre_hip_timers.so")))
    else:
        print(build(verbose=True))
