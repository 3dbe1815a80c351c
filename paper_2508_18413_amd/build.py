"""Builds libpmcmc.so (HIP, gfx950) in-tree from csrc/*.hip with hipcc.

Every source compiles to an object in _build/ (in parallel), then one shared
library is linked next to this file.  Packed FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libpmcmc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PMC_OFFLOAD_ARCH", "gfx950")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"),
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
         "-Rpass-analysis=kernel-resource-usage"]
# Per-source additions.  The wide logistic GEMM's epilogues are fully unrolled
# loops over a lane's 64 accumulator elements; above the compiler's default
# size limit for a requested full unroll the loop stays rolled and the
# accumulators move to private memory.
FILE_FLAGS = {"logreg_wide.hip": ["-mllvm", "-pragma-unroll-threshold=200000"]}
# Every kernel's private segment (spills and private arrays) stays within the
# HIP runtime's default per-thread stack of 1 KiB.
MAX_PRIVATE_BYTES = 1024
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|LDS Size \[bytes/block\]):\s+(\S+)")


def _resources(text: str) -> list[dict]:
    """Per-kernel resource usage from the compiler's kernel-resource-usage remarks."""
    out, cur = [], None
    for line in text.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = {"kernel": val}
            out.append(cur)
        elif cur is not None:
            cur[key.split(" ")[0]] = int(val)
    return out


def _compile(src: str, obj: str) -> tuple[str, int, str, list]:
    cmd = [HIPCC] + FLAGS + FILE_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    text = p.stdout + p.stderr
    res = _resources(text)
    err = "\n".join(l for l in text.splitlines()
                    if "packed-fp32" not in l and "remark:" not in l and not re.match(r"^\s*\d*\s*\|", l))
    return src, p.returncode, err, res


def build(verbose: bool = False) -> str:
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    objs = [os.path.join(bdir, os.path.basename(s) + ".o") for s in srcs]
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    failed, table = [], []
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        for src, rc, err, res in ex.map(lambda so: _compile(*so), zip(srcs, objs)):
            if rc != 0:
                failed.append((src, err))
                continue
            if verbose and err.strip():
                print(err, file=sys.stderr)
            for r in res:
                r["source"] = os.path.basename(src)
                table.append(r)
                if r.get("ScratchSize", 0) > MAX_PRIVATE_BYTES:
                    failed.append((src, f"{r['kernel']}: {r['ScratchSize']} bytes of private memory per lane "
                                        f"(limit {MAX_PRIVATE_BYTES})"))
    with open(os.path.join(bdir, "kernel_resources.txt"), "w") as f:
        f.write("source\tVGPRs\tAGPRs\tscratch_bytes_per_lane\tLDS_static\tkernel\n")
        for r in sorted(table, key=lambda r: (r["source"], r["kernel"])):
            f.write(f"{r['source']}\t{r.get('VGPRs', '')}\t{r.get('AGPRs', '')}\t{r.get('ScratchSize', '')}\t"
                    f"{r.get('LDS', '')}\t{r['kernel']}\n")
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
