"""MI355X-native D3Q27 KBC lattice Boltzmann (arXiv:1507.02518).

The compute path is the HIP library ``libkbc.so`` (sources in ``csrc/``,
C-ABI declared in ``include/kbc.h``); ``kbc`` is its thin ctypes binding and
``inputs`` builds seeded initial velocity fields.  Importing the package does
not load the library; the first call into ``kbc`` does, and fails loudly if
it is missing.
"""
__all__ = ["kbc", "inputs"]
