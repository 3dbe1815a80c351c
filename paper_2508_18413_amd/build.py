"""Builds libpmcmc.so (HIP, gfx950) in-tree from csrc/*.hip with hipcc.

Every source compiles to an object in _build/ (in parallel), then one shared
library is linked next to this file.  Packed FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libpmcmc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PMC_OFFLOAD_ARCH", "gfx950")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"),
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def _compile(src: str, obj: str) -> tuple[str, int, str]:
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32" not in l)
    return src, p.returncode, err


def build(verbose: bool = False) -> str:
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    objs = [os.path.join(bdir, os.path.basename(s) + ".o") for s in srcs]
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    failed = []
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        for src, rc, err in ex.map(lambda so: _compile(*so), zip(srcs, objs)):
            if rc != 0:
                failed.append((src, err))
            elif verbose and err.strip():
                print(err, file=sys.stderr)
    if failed:
        for src, err in failed:
            print(f"--- {src}\n{err}", file=sys.stderr)
        raise RuntimeError("libpmcmc build failed: " + ", ".join(os.path.basename(s) for s, _ in failed))
    tmp = SO + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
