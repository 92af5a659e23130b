"""MI355X-native fused k-means Lloyd iteration.

The compute lives in ``libkmeans_mi355x.so`` (hand-written gfx950 kernels
behind the C ABI of ``include/kmeans_mi355x.h``); ``binding`` is a thin ctypes
layer over it.  Importing the package does not load the library.
"""

__all__ = ["binding", "datagen", "build"]
