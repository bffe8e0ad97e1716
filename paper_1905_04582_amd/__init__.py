"""MI355X-native hot path of Bayesian multidimensional scaling (Holbrook et al.,
"Massive parallelization boosts big Bayesian multidimensional scaling").

The compute lives in the HIP library ``libmassivemds.so`` (C-ABI declared in
``include/massivemds.h``); ``paper_1905_04582_amd.api`` is a thin ctypes
binding over it that uses torch only for device memory and streams.
"""

__all__ = ["api", "synth"]
