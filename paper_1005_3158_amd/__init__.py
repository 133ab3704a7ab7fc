"""MI355X-native explicit finite-element casting-solidification step.

The HIP library (libcastfem.so, built by build.py) holds every step of the
path; `castfem` is its ctypes binding.
"""
from . import castfem  # noqa: F401
