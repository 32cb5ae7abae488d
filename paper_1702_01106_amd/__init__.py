"""MI355X-native implementation of grim's per-zone Newton-Raphson method.

The GPU path lives in ``libgrim.so`` (hand-written HIP for gfx950 behind a
C ABI); :mod:`paper_1702_01106_amd.grim` is its ctypes binding.  Importing the
package loads nothing; the binding loads the library on first use and raises
if it has not been built.
"""
__all__ = ["grim", "workloads"]
