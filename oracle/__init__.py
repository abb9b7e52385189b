"""FP64 CPU oracle for the pressure-projection / velocity-extension Poisson path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP path: the spectral
transforms here are scipy/numpy library routines, and the z direction is
solved by a generalised symmetric eigendecomposition rather than by a
tridiagonal sweep.

What it computes (section 3.2, eqs. for p-hat, the pressure Poisson equation
and the velocity correction; section 3.6, eqs. for the Stefan potential, the
liquid-velocity extension and the interface velocity):

* ``solve``   -- p with L_h p = f - mean_W(f) and sum(dV p) = 0, where L_h is
  the second-order marker-and-cell Laplacian D(G(.)) of section 3;
* ``project`` -- the constant-coefficient split projection step;
* ``extend``  -- the divergence-free liquid-velocity extension and the
  interface velocity;
* ``interface_terms`` -- |grad C| by Youngs' finite differences, the Stefan
  source s and the interface-velocity jump q on faces (sections 3.2, 3.4, 3.6);
* ``advect`` -- the VoF advection of section 3.1 (eqs. cadv, fluxes,
  final_corr_1, final_corr_2) with the MTHINC flux of the method it cites,
  consuming the interface velocity.

Every function names the passage it follows.  Pins against closed forms,
brute-force dense solves and library special cases live in ``tests/``.
"""

from .grid import Grid  # noqa: F401
from .stencils import grad, div, lap, face_density, grad_lower, face_density_lower  # noqa: F401
from .solver import (  # noqa: F401
    solve,
    z_operator_dense,
    eigenvalues_1d,
    assemble_pressure_rhs,
    project,
    extend,
)
from .interface import interface_terms, youngs_gradient  # noqa: F401
from .advection import advect  # noqa: F401
