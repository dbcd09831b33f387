"""MI355X-native Geant4-style gamma navigation (HIP/gfx950) behind a C ABI.

The compute path lives in ``libgnav.so`` (see ``include/gnav.h``); ``gnav``
is its ctypes binding and raises ImportError when the library has not been
built (``python -m paper_1209_5235_amd.build``).  There is no CPU fallback.
"""

_EXPORTS = ("Context", "Tally", "primaries_to_device", "make_log", "log_to_numpy")


def __getattr__(name):
    # The binding is imported on first use so that the build step can run
    # before the library exists.
    if name == "gnav" or name in _EXPORTS:
        import importlib
        mod = importlib.import_module(__name__ + ".gnav")
        return mod if name == "gnav" else getattr(mod, name)
    raise AttributeError(name)
