"""MI355X-native SuperSCS hot path (arXiv 1903.06477).

The solver itself lives in the HIP library ``libsscs`` (sources in ``csrc/``,
C ABI in ``include/sscs.h``); ``sscs`` is its thin Python binding.  Importing
this package loads nothing; the binding loads the library on first use and
raises if it has not been built.
"""
__all__ = ["generators", "sscs"]
