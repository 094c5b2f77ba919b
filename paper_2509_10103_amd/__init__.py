"""MI355X-native hot path of the nonlinear-optimal-perturbation method for
pulsatile pipe flow (Keuchel & Avila, arXiv 2509.10103).

The compute lives in hand-written HIP kernels behind the C ABI declared in
``include/npo.h`` (``libnpo.so``); :mod:`paper_2509_10103_amd.npo` is the thin
ctypes binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
__all__ = ["npo", "synth", "configs"]
