"""Build the BMND HIP library (libbmnd.so) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbmnd.so")
SOURCES = ["host_api.cpp", "host_schedule.cpp", "host_tables.cpp", "kernels.hip",
           "kernels_filter_cube.hip", "kernels_filter_1d.hip", "kernels_match_1d.hip",
           "kernels_match_nd.hip",
           "kernels_match_pois.hip", "host_moments.cpp", "corr_noise.hip", "noalloc.hip",
           "kernels_filter_nd.hip", "kernels_filter_nd_2d_ht.hip", "kernels_filter_nd_2d_wie.hip",
           "kernels_filter_nd_3d_ht.hip", "kernels_filter_nd_3d_wie.hip"]

# Packed FP32 VALU instructions are kept out of the generated code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs, cmds = [], []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src + ".o")
        cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall",
               "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = DEVICE_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    # the translation units compile independently
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 1, 16))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for f in [pool.submit(subprocess.check_call, c, cwd=CSRC) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
