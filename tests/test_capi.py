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
