"""MI355X-native hot path of the cuSZ+ error-bounded lossy compressor.

Submodules:
  ``ebc``   -- thin ctypes binding over the HIP C-ABI library ``libebc.so``
  ``synth`` -- seeded synthetic fields (shared input generators)

Nothing is imported eagerly: importing the package never loads the HIP
library, so the CPU-only tests can use ``synth`` on a machine without a GPU.
"""
__all__ = ["ebc", "synth"]
