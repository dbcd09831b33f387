"""Build libgnav.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1209_5235_amd.build [--verbose]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgnav.so")

# (source, object name, extra defines): the transport kernel is built once per
# track-pool size, again per pool size with sphere sections, and once for
# unrotated boxes.
SOURCES = [("gnav_host.cpp", "gnav_host", ()), ("gnav_kernels.hip", "gnav_kernels", ("GNAV_SPHERES",)),
           ("gnav_mlp.hip", "gnav_mlp", ())] + \
          [("gnav_transport.hip", f"gnav_transport_pool{p}", (f"GNAV_POOL={p}",)) for p in (64, 128, 256)] + \
          [("gnav_transport.hip", f"gnav_transport_pool{p}_spheres", (f"GNAV_POOL={p}", "GNAV_SPHERES"))
           for p in (64, 128, 256)] + \
          [("gnav_transport.hip", "gnav_transport_pool64_axis_boxes", ("GNAV_POOL=64", "GNAV_AXIS_BOXES"))]

# -ffp-contract=off: no fused multiply-add contraction, so each distance is
# rounded operation by operation.  The packed-fp32 feature is disabled for all
# device code.
HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
    "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return h


def build(verbose=False, defines=(), out=None, objdir=None):
    """Compile the sources (in parallel); `defines` adds -D flags, `out` overrides the
    library path and `objdir` the object directory."""
    tmpdir = objdir or os.path.join(HERE, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    objs, procs = [], []
    for src, name, extra in SOURCES:
        obj = os.path.join(tmpdir, name + ".o")
        cmd = [hipcc(), "-x", "hip"] + HIPFLAGS + [f"-D{d}" for d in tuple(defines) + tuple(extra)] + \
              ["-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    target = out or LIB
    tmp = target + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
