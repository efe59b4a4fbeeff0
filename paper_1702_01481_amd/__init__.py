"""MI355X-native hot path of the blocked linear method (arXiv:1702.01481).

The compute path lives in the HIP library ``libblm.so`` (C ABI, declared in
``include/blm.h``); ``paper_1702_01481_amd.blm`` is its thin ctypes binding.
Importing the package does not load the library.
"""
