"""MI355X (gfx950) implementation of one iteration of the kinetostatic
compliance method (KCM) of Protofold II, behind the C ABI of ``libkcm.so``.

``paper_1712_05012_amd.kcm`` is a thin ctypes binding with the ABI's names;
every step of the iteration runs in the HIP kernels of ``csrc/``.  Importing
this package does not load the library; the first call does, and fails
loudly if ``libkcm.so`` has not been built.
"""
