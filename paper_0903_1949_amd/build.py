"""Build libpprt.so in-tree with hipcc for gfx950.

    python -m paper_0903_1949_amd.build      (or __graft_entry__.build())

Every HIP source under csrc/ is compiled with packed-FP32 instructions
disabled and linked into paper_0903_1949_amd/libpprt.so next to this file."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpprt.so")
ARCH = os.environ.get("PPRT_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libpprt)")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object (in parallel), then link the shared
    library.  Always recompiles.  Returns the library path."""
    cc = hipcc()
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [cc, *HIP_FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs[:1]); procs = procs[1:]
    _drain(procs)
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if out.returncode != 0:
        raise RuntimeError("link failed:\n" + out.stdout)
    os.replace(tmp, LIB)
    return LIB


def _drain(procs):
    for src, p in procs:
        text, _ = p.communicate()
        text = text.decode(errors="replace")
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{text}")
        noise = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()
                 and "not a recognized feature" not in l]
        if noise:
            print(f"[{os.path.basename(src)}]\n" + "\n".join(noise), file=sys.stderr)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
