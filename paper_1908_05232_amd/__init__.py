"""MI355X-native hot path of the coupled flood-pedestrian simulator (arXiv 1908.05232).

``paper_1908_05232_amd.fps`` is the ctypes binding of the HIP library
``libfps.so`` (C-ABI declared in ``include/fps.h``); ``inputs`` builds seeded
synthetic scenarios.
"""
