"""MI355X-native all-pairs dynamic time warping (DTW).

The compute path is a HIP library for gfx950 (``csrc/``) behind a C ABI
(``include/dtwmi.h``); ``binding`` is its thin Python wrapper.  ``synth``
makes the seeded synthetic inputs.  Importing this package does not load the
library; ``binding`` loads it on first use and raises if it is missing.
"""
__all__ = ["synth", "binding"]
