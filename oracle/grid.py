"""Grid of the oracle (section 3: fixed Cartesian grid, marker-and-cell layout).

The paper uses a uniform grid.  The z direction may also be stretched
(cell widths dzf[k] given by the caller); x and y stay uniform so that the
constant-coefficient operator keeps its x/y eigen-decomposition.  Distances
between neighbouring cell centres are dzc[k] = (dzf[k] + dzf[k+1]) / 2 for
the face k+1/2; with periodic z the last face wraps to the first cell.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, nx: int, ny: int, nz: int, dx: float, dy: float, dzf, bc: str):
        bc = bc.upper()
        if len(bc) != 3 or any(c not in "PN" for c in bc):
            raise ValueError(f"bc must be 3 letters from P/N, got {bc!r}")
        dzf = np.asarray(dzf, dtype=np.float64).reshape(-1)
        if dzf.shape != (nz,):
            raise ValueError("dzf must have nz entries")
        if bc[2] == "P" and nz < 3:
            raise ValueError("periodic z needs nz >= 3")
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy = float(dx), float(dy)
        self.dzf = dzf
        self.bc = bc
        dzc = np.full(nz, np.nan)
        if nz > 1:
            dzc[:-1] = 0.5 * (dzf[:-1] + dzf[1:])
        if bc[2] == "P":
            dzc[-1] = 0.5 * (dzf[-1] + dzf[0])
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
