"""Build libhistmi.so in-tree for gfx950 with hipcc (kernels + C ABI runtime)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhistmi.so")
LIB_TIMELINE = os.path.join(HERE, "libhistmi_timeline.so")
SOURCES = ["kernels.hip", "noalloc.hip", "api.cpp", "plan.cpp", "server.cpp", "ingest.cpp"]
ARCH = "gfx950"


def hip_flags():
    return [
        "--offload-arch=" + ARCH,
        "-O3",
        "-std=c++17",
        "-fPIC",
        # keep packed-fp32 instructions out of generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
    ]


def _link(objs, out, verbose):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Build libhistmi.so and its diagnostic twin libhistmi_timeline.so (the same sources,
    the kernel compiled with HISTMI_TIMELINE: per-workgroup event timestamps, see
    include/histmi_timeline.h)."""
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(bdir, src + ".o")
        cmd = ["hipcc"] + hip_flags() + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    _link(objs, LIB, verbose)
    tl_obj = os.path.join(bdir, "kernels_timeline.o")
    cmd = ["hipcc"] + hip_flags() + ["-DHISTMI_TIMELINE", "-c", os.path.join(CSRC, "kernels.hip"), "-o", tl_obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    _link([tl_obj if o.endswith("kernels.hip.o") else o for o in objs], LIB_TIMELINE, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
