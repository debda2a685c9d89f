"""MI355X-native Polyhedral Template Matching (arXiv:1603.05143).

``ptm`` is the ctypes binding of the HIP library ``libptm.so`` (C ABI in
``include/ptm.h``); ``synthetic`` builds seeded test and benchmark inputs.
"""
