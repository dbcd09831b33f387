"""The C-ABI library loads and exports every symbol the public header declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gnav.h")
LIB = os.path.join(ROOT, "paper_1209_5235_amd", "libgnav.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gnav_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["gnav_create", "gnav_destroy", "gnav_upload_geometry", "gnav_locate",
                     "gnav_compute_step", "gnav_compute_safety", "gnav_transport_batch",
                     "gnav_read_tallies", "gnav_tally_create"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1209_5235_amd import gnav
    for n in declared_functions():
        assert hasattr(gnav, n), n


def test_no_device_calls_without_gpu_fail_cleanly():
    """Without a visible GPU, gnav_create reports an error instead of crashing."""
    import torch
    if torch.cuda.is_available():
        return
    from paper_1209_5235_amd import gnav
    h = ctypes.c_void_p()
    st = gnav.gnav_create(0, ctypes.byref(h))
    assert st != 0


def _c_layout(struct, fields):
    """sizeof and offsetof of `fields` in `struct`, from a C program built with gcc
    against the public header."""
    import subprocess
    import tempfile
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "gnav.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(src, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


def test_binding_structs_match_the_header_layout():
    """Every ctypes structure of the binding has the size and field offsets of the
    C structure it mirrors (a field added on one side only fails here)."""
    from paper_1209_5235_amd import gnav
    for name in ("gnav_geometry_desc", "gnav_batch", "gnav_step_outputs", "gnav_tuning"):
        cls = getattr(gnav, name)
        fields = [f[0] for f in cls._fields_]
        size, offsets = _c_layout(name, fields)
        assert ctypes.sizeof(cls) == size, name
        assert [getattr(cls, f).offset for f in fields] == offsets, name


def test_record_dtypes_match_the_header_layout():
    """The numpy views of device records (log, digest, crossing) have the C sizes and
    field offsets."""
    from paper_1209_5235_amd import gnav
    for name, dt in (("gnav_logrec", gnav.LOG_DTYPE), ("gnav_digest", gnav.DIGEST_DTYPE),
                     ("gnav_crossing", gnav.CROSSING_DTYPE)):
        fields = list(dt.names)
        size, offsets = _c_layout(name, fields)
        assert dt.itemsize == size, name
        assert [dt.fields[f][1] for f in fields] == offsets, name
