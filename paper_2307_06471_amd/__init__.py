"""MI355X-native compact RKDG (cRKDG) step library: HIP kernels behind a
C ABI (include/crkdg.h), with a thin ctypes binding (crkdg.py)."""
from . import crkdg  # noqa: F401
