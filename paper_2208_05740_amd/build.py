"""Compile the gfx950 HIP library libgcp.so in-tree with hipcc.

Usage:  python -m paper_2208_05740_amd.build
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgcp.so")
ARCH = os.environ.get("GCP_OFFLOAD_ARCH", "gfx950")
SOURCES = ["kernels.hip", "conv_kernels.hip", "chain_kernels.hip", "persist_kernels.hip", "scratch.hip", "gcp_api.cpp", "bab.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed fp32 instructions are left to ordinary float code only
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    obj = os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")
    os.makedirs(os.path.dirname(obj), exist_ok=True)
    extra = ["--cuda-host-only"] if src.endswith(".cpp") else []
    cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=True):
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    # a command-line example that uses the C ABI alone (no Python)
    ex = os.path.join(HERE, "examples", "gcp_bound_mlp")
    cmd = ["hipcc", "-O2", "-std=c++17", os.path.join(HERE, "examples", "gcp_bound_mlp.cpp"), "-L" + HERE, "-lgcp",
           "-Wl,-rpath,$ORIGIN/..", "-o", ex]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"example build failed:\n{r.stderr}")
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
