"""Compile the HIP sources into paper_1502_07442_amd/libngravs.so (gfx950).

Each source is compiled to its own object in parallel (the kernels of one
file never call device code of another), then the objects are linked."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libngravs.so")
SOURCES = ["api.hip", "build.hip", "scan.hip", "sort.hip", "walk.hip", "serve.hip", "short.hip", "pm.hip",
           "noalloc.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    # no packed FP32 instructions: some of their forms have given wrong results on these machines
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    lines = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    return r.returncode, lines


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in srcs]
    cmds = [["hipcc", *FLAGS, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(srcs, objs)]
    if verbose:
        print(" ".join(cmds[0][:-4]) + " -c <each source>", flush=True)
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = False
    for s, (rc, lines) in zip(srcs, results):
        if rc != 0:
            failed = True
            sys.stderr.write(f"{s}:\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed")
    rc, lines = _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"])
    if rc != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError("hipcc link failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
