"""MI355X-native FC(Gram)-based spectral ISPH step.

The compute path is the HIP library ``libfcsph.so`` (sources in ``csrc/``),
reached through the ctypes binding in ``api``.  ``synth`` holds the seeded
manufactured inputs.  Importing this package does not load the library; the
first call into ``api`` does, and it raises if the library is missing.
"""
__all__ = ["api", "synth"]
