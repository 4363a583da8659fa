"""Build libmad.so (HIP for gfx950) in-tree with hipcc.

Run as ``python -m paper_2509_00406_amd.build`` (the repository's build entry point calls the same function).
Every call recompiles (the objects go to _build/ next to the sources).
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libmad.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["kernels_patch.hip", "kernels_eval.hip", "kernels_pattern.hip", "host_mesh.cpp", "host_patch.cpp", "host_layout.cpp",
           "kernels_mlp.hip", "kernels_jac.hip", "layout.cpp", "eval.cpp", "autotune.cpp", "mlp.cpp", "api.cpp",
           "eval_static.hip"]

# -packed-fp32-ops: keep the compiler from forming packed FP32 (v_pk_*_f32) instructions.
# -munsafe-fp-atomics: hardware FP32/FP64 atomic add instead of compare-and-swap loops.
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-pthread", "-I", os.path.join(os.path.dirname(HERE), "include")]


# Element kernels: let the compiler drop arithmetic on the structurally zero channels of the duals
# (x * 0 -> 0 and x + 0 -> x need no-NaN/no-Inf and no-signed-zero assumptions). Their finiteness
# checks read exponent bits (kernels_common.hpp). No reassociation: sums keep their order.
ELEMENT_FLAGS = ["-fno-signed-zeros", "-ffinite-math-only"]
EXTRA = {"kernels_patch.hip": ELEMENT_FLAGS, "kernels_eval.hip": ELEMENT_FLAGS, "kernels_jac.hip": ELEMENT_FLAGS}


def build(verbose: bool = False, jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC, *COMMON, *EXTRA.get(src, []), *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            time.sleep(0.2)
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(f"--- {src} ---\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "-pthread", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
