"""MI355X-native hot path of the transformer density-operator ansatz (arXiv 2502.20723).

The compute lives in the HIP library ``libtdo.so`` (C-ABI declared in
``include/tdo.h``); ``tdo`` is its thin ctypes binding.
"""
