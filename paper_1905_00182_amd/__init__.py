"""MI355X-native immersed-boundary compressible Navier-Stokes solver (Wang, Tian & Lai).

The solver itself is the C-ABI library ``libfsa.so`` built from ``csrc/``; ``fsa`` is its
thin Python binding (argument marshalling only) and ``workloads`` builds seeded inputs.
Nothing is loaded at import time; ``fsa.lib()`` loads the library on first use and raises
if it has not been built.
"""
