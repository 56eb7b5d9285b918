"""MI355X-native hPLMM: two-level multiscale preconditioner (coarse mortar
space + contact-grain smoother) inside right-preconditioned FGMRES for
voxel Q1 linear elasticity.

Importing the package loads nothing native.  ``paper_2509_19777_amd.hplmm``
is the ctypes binding of the HIP library; ``paper_2509_19777_amd.synth`` is
the seeded synthetic-input generator.
"""
