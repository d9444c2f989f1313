"""MI355X-native staggered-grid P_N time step (StaRMAP, arXiv 2004.02833).

The computation lives in libpm.so (HIP for gfx950) behind the C ABI of
include/pm.h; `binding` marshals arguments through ctypes and `autograd`
wraps forward + adjoint as a torch.autograd.Function.
"""
from .binding import *  # noqa: F401,F403
from .binding import EXPORTED, LIB_PATH, PmError, lib  # noqa: F401
