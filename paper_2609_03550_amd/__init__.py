"""MI355X-native quasi-cylindrical direction-splitting (QDS) field advance.

The compute path is the HIP library ``libqds`` (C ABI, see include/qds.h) behind
the thin ctypes binding in ``paper_2609_03550_amd.qds``.  Importing the package
loads nothing; ``paper_2609_03550_amd.qds`` loads the library and raises if it
is missing.
"""
