"""Grid of the oracle (section 3: fixed Cartesian grid, marker-and-cell layout).

The paper uses a uniform grid.  The z direction may also be stretched
(cell widths dzf[k] given by the caller); x and y stay uniform so that the
constant-coefficient operator keeps its x/y eigen-decomposition.  Distances
between neighbouring cell centres are dzc[k] = (dzf[k] + dzf[k+1]) / 2 for
the face k+1/2; with periodic z the last face wraps to the first cell.

Boundary conditions of the pressure (and of the Stefan potential, which
shares them, section 3.6), per direction and end:
  'P' periodic (both ends of a direction),
  'N' wall: zero normal gradient (zero normal velocity),
  'D' outflow: p = 0 on the boundary face (the zero-pressure outflow of the
      cases of section 4); the face lies half a cell from the last centre.
``bc`` is 3 letters (one per direction x, y, z, both ends alike) or 6
letters (x-, x+, y-, y+, z-, z+).  With a 'D' end anywhere the discrete
Laplacian is non-singular and no gauge is fixed.
"""
from __future__ import annotations

import numpy as np


def parse_bc(bc: str):
    """((x-, x+), (y-, y+), (z-, z+)) from 3 or 6 letters of P/N/D."""
    bc = str(bc).upper()
    if len(bc) == 3:
        ends = tuple((c, c) for c in bc)
    elif len(bc) == 6:
        ends = tuple((bc[2 * a], bc[2 * a + 1]) for a in range(3))
    else:
        raise ValueError(f"bc must have 3 or 6 letters, got {bc!r}")
    for lo, hi in ends:
        if lo not in "PND" or hi not in "PND":
            raise ValueError(f"bc letters must be P, N or D, got {bc!r}")
        if (lo == "P") != (hi == "P"):
            raise ValueError(f"a periodic direction is periodic at both ends: {bc!r}")
    return ends


def canonical_bc(ends) -> str:
    """3 letters when both ends of every direction agree, else 6."""
    if all(lo == hi for lo, hi in ends):
        return "".join(lo for lo, _ in ends)
    return "".join(lo + hi for lo, hi in ends)


class Grid:
    def __init__(self, nx: int, ny: int, nz: int, dx: float, dy: float, dzf, bc: str):
        ends = parse_bc(bc)
        dzf = np.asarray(dzf, dtype=np.float64).reshape(-1)
        if dzf.shape != (nz,):
            raise ValueError("dzf must have nz entries")
        if ends[2][0] == "P" and nz < 3:
            raise ValueError("periodic z needs nz >= 3")
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy = float(dx), float(dy)
        self.dzf = dzf
        self.ends = ends
        self.bc = canonical_bc(ends)
        # no Dirichlet end: L_h has the constants as its null space
        self.singular = not any("D" in e for e in ends)
        dzc = np.full(nz, np.nan)
        if nz > 1:
            dzc[:-1] = 0.5 * (dzf[:-1] + dzf[1:])
        if ends[2][0] == "P":
            dzc[-1] = 0.5 * (dzf[-1] + dzf[0])
        elif ends[2][1] == "D":
            dzc[-1] = 0.5 * dzf[-1]  # last centre to the outflow face
        self.dzc = dzc

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def cell_volume(self):
        """dV[k, j, i] = dx dy dzf[k], broadcastable to the field shape."""
        return (self.dx * self.dy) * self.dzf[:, None, None]

    def weighted_mean(self, f):
        dv = self.cell_volume()
        return float((f * dv).sum() / (dv.sum() * self.nx * self.ny))

    @classmethod
    def from_config(cls, cfg):
        return cls(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dzf(), cfg.bc)
