"""MI355X-native hot path of the explicit order-2k generalized-alpha method
with Kronecker-preconditioned mass solves for isogeometric structural
dynamics.  The compute runs in hand-written HIP kernels behind the C ABI of
``include/ga.h``; ``paper_2102_11536_amd.ga`` is the thin ctypes binding.
Importing this package loads nothing; ``ga`` loads the shared library."""
