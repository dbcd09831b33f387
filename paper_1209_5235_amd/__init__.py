"""MI355X-native Geant4-style gamma navigation (HIP/gfx950) behind a C ABI.

The compute path lives in ``libgnav.so`` (see ``include/gnav.h``); ``gnav``
is its ctypes binding.  Build with ``python -m paper_1209_5235_amd.build``.
"""
from . import gnav  # noqa: F401  (fails loudly if libgnav.so is missing)
from .gnav import Context, Tally, primaries_to_device, make_log, log_to_numpy  # noqa: F401
