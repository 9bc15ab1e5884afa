"""MI355X-native WENO-TT hot path: a HIP library (libwenott.so) behind a C ABI
(include/wenott.h) and its ctypes binding (``wenott``)."""
from . import wenott  # noqa: F401
from .wenott import Solver, default_opts  # noqa: F401
