"""Build libnr.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libnr.so")
BUILD_DIR = os.path.join(PKG, "_build")

SOURCES = ["nr_api.hip", "nr_kernels_f64.hip", "nr_kernels_f32.hip", "nr_integrators.hip",
           "nr_hmc.hip", "nr_vi_mvn.hip", "nr_kernels_scan.hip", "nr_autotune.hip"]
# compiled once per (precision, deep bucket); the bucket list is read from
# the NR_BUCKETS_DEEP macro so it cannot drift from the C++ side
BUCKET_SOURCE = "nr_kernels_bucket.hip"


def deep_buckets():
    text = open(os.path.join(CSRC, "nr_internal.hpp")).read()
    m = re.search(r"#define NR_BUCKETS_DEEP\(X\)((?:\s*X\(\d+\))+)", text)
    if not m:
        raise RuntimeError("NR_BUCKETS_DEEP not found in nr_internal.hpp")
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


# Translation units whose kernels are scheduled for instruction-level
# parallelism (LLVM's max-ILP machine scheduler) rather than for occupancy:
# the deep buckets (one wave per SIMD in FP64, where nothing but the wave's
# own independent work hides latency) and the FP32 kernels.  Measured on
# MI355X: ragged 16384-item batch 42.2 -> 40.9 ms in FP64 and 30.2 -> 29.6 ms
# in FP32, 4096-draw FP32 batch 1.53 -> 1.49 ms, results bitwise unchanged;
# the two-wave FP64 kernels of 1-12 layers gained nothing and keep the default.
ILP_SOURCES = (BUCKET_SOURCE, "nr_kernels_f32.hip")
ILP_FLAGS = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]


def tu_flags(src: str) -> list:
    """Compiler flags of one translation unit beyond FLAGS."""
    return list(ILP_FLAGS) if src in ILP_SOURCES else []


def _compile(job) -> str:
    src, defines, tag = job
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + tag + ".o")
    cmd = [HIPCC, *FLAGS, *tu_flags(src), *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = [(src, [], "") for src in SOURCES]
    # the deepest (slowest) buckets first
    for lm in sorted(deep_buckets(), reverse=True):
        for prec in ("F64", "F32"):
            jobs.append((BUCKET_SOURCE, [f"-DNR_PREC={prec}", f"-DNR_BUCKET_LMAX={lm}"],
                         f"_{prec}_{lm}"))
    jobs.sort(key=lambda j: 0 if j[0] == BUCKET_SOURCE else 1)
    workers = max(1, min(len(jobs), os.cpu_count() or 4))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
