"""MI355X-native layered-media linearized Poisson-Boltzmann FMM.

The compute path lives in the HIP/C-ABI library ``liblpbfmm.so`` (sources in
``csrc/``, declarations in ``include/lpb.h``); ``lpb`` is its thin ctypes
binding.  Importing this package does not load the library; ``lpb.load()``
does, and fails loudly when it is missing.
"""
