"""MI355X (gfx950) Vecchia Gaussian log-CDF library: C ABI in include/vecchia.h,
HIP kernels in csrc/, ctypes binding in vecchia.py."""
from . import vecchia  # noqa: F401
