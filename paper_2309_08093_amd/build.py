"""Build libttsketch.so (HIP, gfx950) in-tree with hipcc.

Every translation unit under csrc/ is compiled for gfx950 with packed FP32
instructions disabled, then linked into one shared library next to this file.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libttsketch.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj, r.stderr


def _fresh(src, headers_mtime):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    return os.path.exists(obj) and os.path.getmtime(obj) > max(os.path.getmtime(src), headers_mtime)


def build(verbose=False, jobs=8, incremental=False):
    """Compile every source (or, with incremental=True, only those newer than
    their object or than any header) and link the library."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    hdr = max(os.path.getmtime(h) for h in glob.glob(os.path.join(CSRC, "*.h")) +
              [os.path.join(os.path.dirname(HERE), "include", "tt_sketch.h")])
    todo = [s for s in srcs if not (incremental and _fresh(s, hdr))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        done = dict(zip(todo, ex.map(_compile, todo)))
    results = [done.get(s, (os.path.join(OBJ, os.path.basename(s) + ".o"), "")) for s in srcs]
    if verbose:
        for obj, err in results:
            if err.strip():
                sys.stderr.write(err)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp, *[o for o, _ in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
