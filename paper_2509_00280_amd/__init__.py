"""MI355X-native sparse MTTKRP / CP-ALS over bit-interleaved linearized COO tensors.

The compute path is the HIP library ``libspt.so`` behind the C-ABI declared
in ``include/spt.h``; ``paper_2509_00280_amd.spt`` is its thin ctypes binding.
Importing this package loads nothing: the library is opened on first use and
every entry point fails loudly when it is missing.
"""
__all__ = ["spt", "synth"]
