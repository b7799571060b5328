"""Nystrom kernel filtering (bilateral / nonlocal means) on MI355X.

The filter itself lives in the HIP library ``_lib/libnkf.so`` (C ABI in
``include/nkf.h``); ``paper_1901_06112_amd.nkf`` is the Python binding and
``paper_1901_06112_amd.synth`` draws seeded synthetic workloads.  Importing
this package loads neither torch nor the library.
"""
__all__ = ["nkf", "synth"]
