"""Physical constants (CODATA 2018 exact / recommended values), SI units.

Test infrastructure: part of the FP64 oracle.
"""

C = 299792458.0               # speed of light [m/s]
QE = 1.602176634e-19          # elementary charge [C]
ME = 9.1093837015e-31         # electron mass [kg]
EPS0 = 8.8541878128e-12       # vacuum permittivity [F/m]
HBAR = 1.054571817e-34        # reduced Planck constant [J s]
KB = 1.380649e-23             # Boltzmann constant [J/K]
NA = 6.02214076e23            # Avogadro constant [1/mol]
AMU = 1.66053906660e-27       # atomic mass unit [kg]
