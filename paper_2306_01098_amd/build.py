"""Builds the gfx950 HIP library ``libhisq.so`` in-tree (next to this file).

Every translation unit under ``csrc/`` is compiled by ``hipcc`` for gfx950
into ``_build/`` at the repository root, in parallel, then linked into one
shared library.  hipcc cross-compiles, so no GPU is needed to build.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhisq.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions: plain FP32 arithmetic only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile and link ``libhisq.so``; returns its path.  Raises on failure."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    pending = []
    objs = []
    for src in sources():
        obj = os.path.join(BUILD_DIR, src + ".o")
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        pending.append((src, cmd))
    running = []
    failures = []

    def reap(block: bool):
        for item in list(running):
            src, proc = item
            if block or proc.poll() is not None:
                out, _ = proc.communicate()
                running.remove(item)
                text = out.decode(errors="replace")
                # the host pass does not know the packed-FP32 feature: harmless
                text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
                if proc.returncode != 0:
                    failures.append((src, text))
                elif verbose and text.strip():
                    print(text, file=sys.stderr)

    while pending or running:
        while pending and len(running) < jobs:
            src, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if running:
            running[0][1].wait()
            reap(False)
    if failures:
        msg = "\n".join(f"--- {s}\n{t}" for s, t in failures)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB + ".tmp"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout.decode(errors="replace"))
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
