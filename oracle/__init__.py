"""Plain FP64 CPU oracle for one RK3 / implicit-viscous substep of the
Taylor--Couette DNS of Pirro & Quadrio, "Direct Numerical Simulation of
turbulent Taylor--Couette flow".

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constant generators); the
two sides only ever meet through the seeded input generator, which holds none
of the method's arithmetic.

What it computes (paper section / equation it follows):

* ``grid``     -- geometry, units, radial grid, Fourier domain and wavenumbers
                  (Sec. 2 and Fig. 1; Sec. 4 for the domain; Appendix for the
                  wavenumbers).
* ``compact``  -- fourth-order explicit compact finite-difference
                  coefficients on a 5-point stencil of arbitrarily spaced
                  points (Sec. 2.1; Appendix).
* ``spectral`` -- Fourier transforms and 3/2-rule dealiased products
                  (Appendix: the nonlinear terms HU, HV, HW).
* ``equations``-- velocity recovery from (v, eta) through continuity, the
                  right-hand sides of eq. (final-v) and eq. (final-eta), and
                  the mean (0,0) mode (Sec. 4; Appendix).
* ``stepper``  -- the 3-substep low-storage Runge--Kutta / Crank--Nicolson
                  substep (Sec. 2.1; Sec. 3.1; Sec. 4).
* ``stats``    -- torque (eq. (torque), Table 2), wall shear, Re_tau (Sec. 5),
                  kinetic energy and radial profiles.

Every function is FP64 and vectorised only over Fourier modes; there is no
blocking, fusion or reordering beyond the definitions it follows.  Where the
paper is silent the reading taken is stated in the function's docstring.
"""

from .grid import Geometry, Discretisation
from .compact import compact_coefficients
from .stepper import Oracle

__all__ = ["Geometry", "Discretisation", "compact_coefficients", "Oracle"]
