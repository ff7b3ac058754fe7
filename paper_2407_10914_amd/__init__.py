"""MI355X-native colour-gradient lattice Boltzmann time step (arXiv:2407.10914).

The compute path is the HIP library ``libcglbm.so`` behind the C-ABI declared in
``include/cg_lbm.h``; this package is its thin ctypes binding.
"""
