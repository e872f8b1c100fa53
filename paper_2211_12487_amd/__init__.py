"""MI355X-native TT-ICE: incremental tensor-train updates on gfx950.

The compute lives in the C-ABI library ``libttice.so`` (hand-written HIP
kernels plus a C++ host engine); ``ttice`` is its thin ctypes binding and
``synth`` the seeded input generators."""
