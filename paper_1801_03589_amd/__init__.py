"""MI355X-native NESA EFIE matrix-vector product and GMRES solver.

The compute path is the HIP library ``libnesa.so`` (built by ``build.py``);
``nesa`` is a thin ctypes binding to its C ABI (``include/nesa.h``).
"""
from . import nesa  # noqa: F401
