"""Build libwlra.so (hipcc, gfx950) in-tree next to this file.

Each HIP source is compiled to an object file in parallel (every kernel is
launched from its own translation unit), then the objects are linked into
the shared library."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwlra.so")
SOURCES = ["wlra_api.hip", "k_stream.hip", "k_small.hip", "k_eig.hip", "k_eigmw.hip",
           "k_learn.hip"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-pthread",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unused-value"]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="wlra_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.splitext(f)[0] + ".o") for f in SOURCES]
        cmds = [[hipcc, *FLAGS, "-c", os.path.join(CSRC, f), "-o", o]
                for f, o in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            procs = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for c, p in zip(cmds, procs):
            err = "\n".join(ln for ln in p.stderr.splitlines() if "packed-fp32-ops" not in ln)
            if err.strip() and (verbose or p.returncode != 0):
                print(err, file=sys.stderr, flush=True)
            if p.returncode != 0:
                raise subprocess.CalledProcessError(p.returncode, c)
        tmp = LIB + ".tmp"
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
