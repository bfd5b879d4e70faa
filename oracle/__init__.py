"""FP64 CPU oracle for the laser-dielectric PIC hot path (arXiv 2502.13695).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
link this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP path: the only thing the
two sides have in common is the seeded workload description in ``workloads``.

It is a plain, slow, obviously correct implementation written from the paper:

* ``keldysh``   -- Keldysh photoionization rate, Sec. 2.1 Eq. (1)-(3), with the
  complete elliptic integrals by the arithmetic-geometric mean and the Dawson
  integral by Rybicki's method; evaluated in situ per particle as the paper
  does (Sec. 2.1, footnote on the tabulated elliptic integrals).
* ``philox``    -- counter-based Philox generator (Salmon et al., SC'11), used
  for the Monte-Carlo ionization draws and the neutral loading.
* ``problem``   -- the discrete problem a configuration defines: time step
  (Sec. 3.1, 0.95 of the CFL limit), materials and reduced mass (Sec. 3.2,
  Table 1), geometry of the optical region (Sec. 2.3), laser pulse and its
  fluence (Sec. 3).
* ``pic``       -- the particle-in-cell time step: Yee FDTD with a spatially
  varying permittivity (Sec. 2.3), first-order outflow boundaries with the
  laser injected as a boundary condition (Sec. 3, 3.1), shape-function gather,
  relativistic Boris push, Esirkepov charge-conserving deposit, the one-cycle
  rolling amplitude window (Sec. 2.1, last paragraph) and Monte-Carlo single
  ionization with electron / positive-carrier birth (Sec. 2.1, 3.2).

Parity status of every function is listed in its module header.
"""

from . import constants, keldysh, philox, problem, pic  # noqa: F401
