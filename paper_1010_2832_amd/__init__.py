"""MI355X (gfx950) implementation of one backward-Euler step of the
variational finite-difference method for time-dependent, variable
coefficient Stokes flow on irregular domains: HIP kernels behind the C ABI
in include/vfstokes.h, with a thin ctypes binding (``vfstokes``)."""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvfstokes.so")


def binding():
    """Import the ctypes binding (raises ImportError if the library is not built)."""
    from . import vfstokes
    return vfstokes
