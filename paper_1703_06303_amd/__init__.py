"""MI355X-native sWLR solver (Dutta & Li, arXiv 1703.06303): a C-ABI library
of hand-written gfx950 HIP kernels (libwlra.so) and its ctypes binding."""
from . import wlra  # noqa: F401
