"""MI355X-native hybrid lattice-Boltzmann / finite-difference step for
nematic liquid crystals (Coelho, Araujo, Telo da Gama, arXiv:1907.13415).

The step runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/lc.h``; ``paper_1907_13415_amd.lc`` is a thin ctypes binding with
the same names.  ``paper_1907_13415_amd.inputs`` builds seeded initial states.
"""
