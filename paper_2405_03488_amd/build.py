"""Build libsgpm.so (HIP kernels for gfx950 + C++ host library) in-tree."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(ROOT, "_build")
SO = os.path.join(HERE, "libsgpm.so")
ARCH = os.environ.get("SGPM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "gs.cpp", "host_graph.cpp", "host_pattern.cpp", "host_stats.cpp", "ns_kernels.hip",
           "gs_kernels.hip", "probe_kernels.hip", "batch.cpp", "batch_kernels.hip",
           "model.cpp", "mlp_kernels.hip", "hybrid.cpp", "cost_model.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-command-line-argument",
          f"-I{os.path.join(ROOT, 'include')}"]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = SO + ".tmp"
    # every symbol must resolve at link time, not at the first dlopen
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SO)
    if verbose:
        print(SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
