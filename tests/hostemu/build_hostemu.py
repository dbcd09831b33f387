"""Build the host-emulation copy of the HIP library (a checking tool for tests).

The library's own sources (the same list and defines as the HIP build) are
compiled as C++ for the CPU against tests/hostemu/hip/hip_runtime.h, with
array-bounds checks that trap, and linked with the emulation runtime into
`<out>/libgnav.so`, next to a copy of the ctypes binding (`<out>/gnav.py`,
which loads the library beside it).  Device buffers get guard pages (see
hostemu_rt.cpp).  Two lines of the sources change in the copy: the
GPU-assembly zero of the network's weight addressing becomes an equally opaque
zero for the host compiler, and an out-of-line function defined in a header
gets inline linkage (each GPU code object holds its own copy; a host library
holds one).

Usage: python tests/hostemu/build_hostemu.py [out_dir]
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1209_5235_amd")
CSRC = os.path.join(PKG, "csrc")
DEFAULT_OUT = os.path.join(ROOT, "_build_hostemu")

# (file, text in the library's source, text in the CPU copy)
HOST_PATCHES = [
    ("gnav_learned.h", 'asm volatile("v_mov_b32 %0, 0" : "=v"(z));', 'z = 0;\n  asm volatile("" : "+r"(z));'),
    # out-of-line function defined in a header: one definition per GPU code
    # object, but a shared one on the host
    ("gnav_device.h", "__device__ __attribute__((noinline)) int sph_inside(",
     "__device__ inline __attribute__((noinline)) int sph_inside("),
]

FLAGS = ["-x", "c++", "-std=c++17", "-O1", "-g", "-fPIC", "-pthread", "-ffp-contract=off",
         "-fsanitize=array-bounds", "-fsanitize-trap=array-bounds", "-fno-omit-frame-pointer",
         "-DGNAV_TRANSPORT_WAVES=0",
         "-Wno-unknown-attributes", "-Wno-unused-function", "-Wno-unused-variable",
         "-Wno-ignored-attributes", "-Wno-unused-command-line-argument"]


def compiler():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("clang++ not found")


def _sources():
    sys.path.insert(0, ROOT)
    from paper_1209_5235_amd import build as hipbuild
    return hipbuild.SOURCES


def _digest(patches):
    h = hashlib.sha256()
    for d in (CSRC, HERE, os.path.join(HERE, "hip"), os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            p = os.path.join(d, f)
            if os.path.isfile(p) and f.endswith((".h", ".hip", ".cpp", ".py")):
                h.update(f.encode())
                with open(p, "rb") as fh:
                    h.update(fh.read())
    with open(os.path.join(PKG, "gnav.py"), "rb") as fh:
        h.update(fh.read())
    h.update(repr(patches).encode())
    return h.hexdigest()[:16]


def build(out=None, extra_patches=(), jobs=8, verbose=False):
    """Build (or reuse) the emulation library; returns the output directory."""
    out = out or DEFAULT_OUT
    patches = list(HOST_PATCHES) + list(extra_patches)
    tag = _digest(patches)
    stamp = os.path.join(out, "STAMP")
    if os.path.exists(stamp) and open(stamp).read().strip() == tag and \
            os.path.exists(os.path.join(out, "libgnav.so")):
        return out
    src = os.path.join(out, "src")
    obj = os.path.join(out, "obj")
    os.makedirs(src, exist_ok=True)
    os.makedirs(obj, exist_ok=True)
    for f in os.listdir(CSRC):
        if f.endswith((".h", ".hip", ".cpp")):
            shutil.copy(os.path.join(CSRC, f), os.path.join(src, f))
    for f, old, new in patches:
        p = os.path.join(src, f)
        text = open(p).read()
        if text.count(old) != 1:
            raise RuntimeError(f"host patch of {f} no longer applies: {old!r}")
        open(p, "w").write(text.replace(old, new))
    cxx = compiler()
    cmds = []
    for s, name, extra in _sources():
        cmds.append([cxx] + FLAGS + [f"-D{d}" for d in extra] +
                    ["-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", src, "-c", os.path.join(src, s),
                     "-o", os.path.join(obj, name + ".o")])
    cmds.append([cxx] + FLAGS + ["-I", HERE, "-c", os.path.join(HERE, "hostemu_rt.cpp"),
                                 "-o", os.path.join(obj, "hostemu_rt.o")])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"host-emulation compile failed: {' '.join(cmd)}\n{r.stderr[-4000:]}")

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(run, cmds))
    objs = [c[-1] for c in cmds]
    lib = os.path.join(out, "libgnav.so")
    subprocess.run([cxx, "-shared", "-pthread", "-fsanitize=array-bounds", "-fsanitize-trap=array-bounds",
                    "-o", lib + ".tmp"] + objs, check=True)
    os.replace(lib + ".tmp", lib)
    shutil.copy(os.path.join(PKG, "gnav.py"), os.path.join(out, "gnav.py"))
    with open(stamp, "w") as fh:
        fh.write(tag + "\n")
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else None, verbose=True))
