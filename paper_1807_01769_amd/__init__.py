"""MI355X-native pseudo-spectral Navier-Stokes RK4 step (periodic box, 2D/3D).

The compute path is the HIP library ``libfs.so`` behind the C ABI declared in
``include/fs.h``; ``paper_1807_01769_amd.fs`` is its thin ctypes binding and
raises at import time when the library is missing.  ``inputs`` builds seeded
initial states and has no dependency on the library.
"""
