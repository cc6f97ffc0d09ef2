"""MI355X-native axisymmetric thermal lattice Boltzmann LES (D2Q9 + D2Q4).

Importing the package loads nothing; the HIP library is loaded on first use
of the binding (``paper_1002_3028_amd.lbm``).
"""
