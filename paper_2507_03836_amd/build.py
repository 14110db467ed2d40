"""Build libfhash.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfhash.so")
SOURCES = ["fused_train.hip", "fused_train16.hip", "fused_bwd.hip", "fused_bwd16.hip", "fused.hip",
           "fused_fwd16.hip", "mlp.hip", "api.cpp",
           "index.hip",
           "encode.hip", "optim.hip", "lazy.hip", "sampler.hip", "render.hip", "sort.hip", "coreset.hip", "static_ws.hip",
           "coarse.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("FHASH_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


# Measurement probe (not part of the library): the chip's scattered-access
# ceiling that the fine-level gathers and atomics are held against.
PROBE_SRC = os.path.join(HERE, "probe", "random_access.hip")
PROBE = os.path.join(HERE, "probe", "random_access")


def _probe() -> str:
    cmd = [HIPCC, *[f for f in FLAGS if f != "-fPIC"], PROBE_SRC, "-o", PROBE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for the probe:\n{r.stderr}")
    return PROBE


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        probe = ex.submit(_probe)
        objs = list(ex.map(_compile, SOURCES))
        probe.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
