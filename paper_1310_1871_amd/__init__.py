"""MI355X-native axisymmetric Shan–Chen lattice Boltzmann (arXiv:1310.1871).

The method runs in the HIP library ``liblbm_axi.so`` built from ``csrc/``;
``lbm_axi`` is its ctypes binding.
"""
