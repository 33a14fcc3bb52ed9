"""Build the HIP shared library in-tree with hipcc (gfx950).

``python -m paper_1806_10599_amd.build`` compiles every source under
``csrc/`` to an object file and links ``libpaper_1806_10599_amd.so`` next to
this file.  Objects go to ``_build/`` at the repository root.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBNAME = "libpaper_1806_10599_amd.so"
LIBPATH = os.path.join(HERE, LIBNAME)
ARCH = os.environ.get("RVE_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-I", os.path.join(ROOT, "include"), "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable"]
# no packed FP32 instructions in device code
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
                 shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src: str, obj: str, verbose: bool) -> str:
    cmd = [hipcc(), *COMMON]
    if src.endswith(".hip"):
        cmd += DEVICE_ONLY
    cmd += ["-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = (res.stdout + res.stderr).strip()
    lines = [ln for ln in out.splitlines()
             if "packed-fp32-ops" not in ln and "warnings generated" not in ln]
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n" + "\n".join(lines))
    return "\n".join(lines) if verbose else ""


def build(verbose: bool = False, jobs: int | None = None) -> str:
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(bdir, os.path.basename(s) + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        for msg in ex.map(lambda so: _compile(so[0], so[1], verbose),
                          zip(srcs, objs)):
            if msg:
                print(msg, file=sys.stderr)
    tmp = LIBPATH + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs,
           "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed\n" + res.stdout + res.stderr)
    os.replace(tmp, LIBPATH)
    return LIBPATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
