"""MI355X-native per-step update of the fully discrete third-order Active Flux method for
the 2D Euler equations (Chudzik, Helzel, Porfetye, arXiv 2508.06273).

The compute path is the HIP library ``libaf.so`` built from ``csrc/``; ``af`` is its thin
ctypes binding.  Importing the package loads nothing; ``af`` loads the library on first use
and raises if it has not been built.
"""
__all__ = ["inputs", "af"]
