"""Builds libmbc.so (host planner + C ABI + gfx950 kernels) in-tree with hipcc.

    python -m paper_2201_04269_amd.build      (or call build())

Every source is compiled to an object of its own (in parallel), then linked.
Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (-target-feature -packed-fp32-ops).  The factored
FP32-comp dS kernel of the (5, 4) family (kernels_ds_5_4.hip) is scheduled
with the AMDGPU backend's iterative ILP strategy, which keeps more of its LDS
gathers in flight at its register limit.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
OBJDIR = os.path.join(LIBDIR, "obj")
LIB = os.path.join(LIBDIR, "libmbc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["index_set.cpp", "block_set.cpp", "plan.cpp", "debug_eval.cpp", "abi.cpp", "kernels.hip", "kernels_bwd.hip",
           "kernels_ds_5_4.hip", "blocks.hip", "egraph.cpp", "egraph_exec.hip", "factor_tree.cpp", "factor_tree.hip"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# per-source extra flags
SOURCE_FLAGS = {"kernels_ds_5_4.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]}
LINK = ["-shared", "-fPIC", "--offload-arch=gfx950"]


def source_hash():
    """SHA-256 (first 16 hex digits) of the sources the device code is built
    from and of the per-source compiler flags."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    h.update(repr(sorted(SOURCE_FLAGS.items())).encode())
    return h.hexdigest()[:16]


def _compile(src, verbose):
    obj = os.path.join(OBJDIR, src + ".o")
    cmd = [HIPCC] + FLAGS + SOURCE_FLAGS.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return obj, r


def build(verbose=False, jobs=None):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    failed = [(o, r) for o, r in results if r.returncode != 0]
    for o, r in failed:
        sys.stderr.write(r.stdout + r.stderr)
    if failed:
        raise RuntimeError("hipcc failed building libmbc.so: " + ", ".join(os.path.basename(o) for o, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + LINK + [o for o, _ in results] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libmbc.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
