"""Seeded synthetic inputs for the Poisson / projection / extension path.

This package is shared by the CPU oracle, the GPU tests, ``smoke()`` and
``bench.py``.  It holds none of the method's arithmetic (no divergence,
gradient, Laplacian or Poisson solve): only grids handed to both sides as
inputs, seeded random fields and the recipes that shape them (a smoothed
VoF sphere, a discretely solenoidal velocity built as a curl, a source term
concentrated at the interface).

Array convention used everywhere: float64 numpy arrays shaped
``(nz, ny, nx)`` (C order, so x is the fastest index).  Velocities live on
the faces of a marker-and-cell grid (the staggered arrangement of section
3): ``u[k, j, i]`` sits on face i+1/2, ``v[k, j, i]`` on face j+1/2 and
``w[k, j, i]`` on face k+1/2.  With wall (Neumann) boundaries in a
direction, the face with the last index in that direction is the wall and
holds zero; the face at -1/2 is implicit and also zero.
"""

from .fields import (  # noqa: F401
    uniform_dz,
    stretched_dz,
    cell_centres,
    z_centres,
    gaussian_field,
    remove_weighted_mean,
    random_faces,
    sphere_vof,
    grad_mag_central,
    interface_normal_faces,
    solenoidal_faces,
    Config,
    config,
    CONFIGS,
)
