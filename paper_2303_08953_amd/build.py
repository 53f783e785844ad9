"""Build the HIP library libsgm.so for gfx950 (in-tree, next to this file).

Run as `python -m paper_2303_08953_amd.build` or through
`__graft_entry__.build()`.  Every source under csrc/ is compiled with hipcc
for --offload-arch=gfx950 and linked into one shared library.  Packed FP32
VALU forms are disabled for device code.  Each source's gfx950 assembly is
also emitted (and discarded): printing it checks every instruction's operand
classes, which the object writer does not, so an instruction the compiler
formed with an illegal operand fails the build instead of being encoded.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsgm.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["matrix.hip", "spmv.hip", "tsq.hip", "small.hip", "shifts.hip",
           "ilu.hip", "solver.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
                 shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool, resource_usage: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if resource_usage:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = (r.stdout + r.stderr)
    out = "\n".join(l for l in out.splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if verbose and out.strip():
        print(out)
    return obj


def _check_asm(src: str) -> None:
    out = os.path.join(BUILD, os.path.splitext(src)[0] + ".s")
    cmd = [hipcc(), *[f for f in FLAGS if f != "-fPIC"], "--cuda-device-only",
           "-S", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l)
        raise RuntimeError(f"gfx950 assembly of {src} failed:\n{msg}")
    os.remove(out)


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(2 * len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        checks = [ex.submit(_check_asm, s) for s in SOURCES]
        objs = list(ex.map(lambda s: _compile(s, verbose, resource_usage),
                           SOURCES))
        for c in checks:
            c.result()
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv,
                resource_usage="--usage" in sys.argv))
