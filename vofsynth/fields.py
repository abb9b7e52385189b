"""Seeded synthetic fields and grids (inputs only, none of the method's arithmetic).

Everything here is an *input recipe*.  The paper measures its solver on no
public data set; these fields stand in for the workloads of its section 4
(a smoothed VoF droplet, a velocity field, an interfacial phase-change
source) at the sizes the benchmark configurations name.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_BC_LETTERS = ("P", "N", "D")


def _check_bc(bc: str) -> str:
    """The upper-end letter of each direction (x, y, z) from 3 letters (both
    ends alike) or 6 (x-, x+, y-, y+, z-, z+) of P/N/D: the stored last face
    of each direction is that end's face."""
    bc = bc.upper()
    if len(bc) == 3:
        pairs = [(c, c) for c in bc]
    elif len(bc) == 6:
        pairs = [(bc[2 * a], bc[2 * a + 1]) for a in range(3)]
    else:
        raise ValueError(f"bc must be 3 or 6 letters from P/N/D, got {bc!r}")
    for lo, hi in pairs:
        if lo not in _BC_LETTERS or hi not in _BC_LETTERS or (lo == "P") != (hi == "P"):
            raise ValueError(f"bad bc {bc!r}")
    return "".join(hi for _, hi in pairs)


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------
def uniform_dz(nz: int, lz: float = 1.0) -> np.ndarray:
    """Cell widths of a uniform z grid (the regular grid of section 3)."""
    return np.full(nz, lz / nz, dtype=np.float64)


def stretched_dz(nz: int, lz: float = 1.0, beta: float = 1.5) -> np.ndarray:
    """Cell widths of a symmetric tanh-clustered z grid.

    Face positions z_f[k] = (lz/2) * (1 + tanh(beta*(2k/nz - 1)) / tanh(beta)),
    k = 0..nz, cluster cells at both walls.  The paper only uses uniform grids;
    this wall-clustered grid is the stretched-z workload of the 512x512x256
    benchmark configuration.
    """
    k = np.arange(nz + 1, dtype=np.float64)
    zf = 0.5 * lz * (1.0 + np.tanh(beta * (2.0 * k / nz - 1.0)) / np.tanh(beta))
    zf[0], zf[-1] = 0.0, lz
    return np.diff(zf)


def cell_centres(n: int, h: float) -> np.ndarray:
    """Centres (i + 1/2) h of a uniform direction."""
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def z_centres(dzf: np.ndarray) -> np.ndarray:
    zf = np.concatenate([[0.0], np.cumsum(dzf)])
    return 0.5 * (zf[:-1] + zf[1:])


# ----------------------------------------------------------------------------
# random fields
# ----------------------------------------------------------------------------
def gaussian_field(shape, seed: int) -> np.ndarray:
    """N(0,1) cell-centred field from ``numpy.random.default_rng(seed)``."""
    return np.random.default_rng(seed).standard_normal(size=tuple(shape))


def remove_weighted_mean(f: np.ndarray, dzf: np.ndarray) -> np.ndarray:
    """Subtract the cell-volume-weighted mean (weights dzf along z)."""
    wz = np.asarray(dzf, dtype=np.float64)[:, None, None]
    return f - (f * wz).sum() / (wz.sum() * f.shape[1] * f.shape[2])


def _zero_walls(u, v, w, bc):
    if bc[0] == "N":
        u[:, :, -1] = 0.0
    if bc[1] == "N":
        v[:, -1, :] = 0.0
    if bc[2] == "N":
        w[-1, :, :] = 0.0
    return u, v, w


def random_faces(shape, seed: int, bc: str):
    """Face velocities (u, v, w) ~ N(0,1); wall faces set to zero."""
    bc = _check_bc(bc)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(size=tuple(shape))
    v = rng.standard_normal(size=tuple(shape))
    w = rng.standard_normal(size=tuple(shape))
    return _zero_walls(u, v, w, bc)


# ----------------------------------------------------------------------------
# droplet recipe (the settling / evaporating droplet of section 4)
# ----------------------------------------------------------------------------
def sphere_vof(nx, ny, nz, dx, dy, dzf, seed: int, radius: float = 0.2,
               width_cells: float = 1.5, lo: float = 0.3, hi: float = 0.7):
    """Smoothed VoF indicator of a sphere, C = 1/2 (1 - tanh((r - R) / (w dx))).

    The centre is drawn uniformly from [lo, hi]^3 (in units of the domain
    length along each axis) with ``default_rng(seed)``.  Returns (C, centre).
    """
    rng = np.random.default_rng(seed)
    lx, ly, lz = nx * dx, ny * dy, float(np.sum(dzf))
    c = rng.uniform(lo, hi, size=3) * np.array([lx, ly, lz])
    x = cell_centres(nx, dx)[None, None, :]
    y = cell_centres(ny, dy)[None, :, None]
    z = z_centres(np.asarray(dzf, dtype=np.float64))[:, None, None]
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    C = 0.5 * (1.0 - np.tanh((r - radius * lx) / (width_cells * dx)))
    return C, c


def _centred_diff(a, axis, h_minus_plus, bc_letter):
    """(a[+1] - a[-1]) / distance, periodic wrap or mirrored ghost at walls."""
    if bc_letter == "P":
        ap = np.roll(a, -1, axis=axis)
        am = np.roll(a, 1, axis=axis)
    else:
        n = a.shape[axis]
        idx_p = np.minimum(np.arange(n) + 1, n - 1)
        idx_m = np.maximum(np.arange(n) - 1, 0)
        ap = np.take(a, idx_p, axis=axis)
        am = np.take(a, idx_m, axis=axis)
    return (ap - am) / h_minus_plus


def _centre_spacings(dzf, periodic):
    """Distance between centres k-1 and k+1 (mirror ghosts at walls)."""
    dzf = np.asarray(dzf, dtype=np.float64)
    if periodic:
        dm, dp = np.roll(dzf, 1), np.roll(dzf, -1)
    else:
        dm = np.concatenate([[dzf[0]], dzf[:-1]])
        dp = np.concatenate([dzf[1:], [dzf[-1]]])
    return 0.5 * dm + dzf + 0.5 * dp


def grad_mag_central(C, dx, dy, dzf, bc: str):
    """|grad C| at cell centres by central differences (an input recipe).

    Returns (|grad C|, (gx, gy, gz)).  The paper's Youngs stencil is not
    specified; this plain central difference only shapes the synthetic source.
    """
    bc = _check_bc(bc)
    gx = _centred_diff(C, 2, 2.0 * dx, bc[0])
    gy = _centred_diff(C, 1, 2.0 * dy, bc[1])
    hz = _centre_spacings(dzf, bc[2] == "P")[:, None, None]
    gz = _centred_diff(C, 0, hz, bc[2])
    return np.sqrt(gx * gx + gy * gy + gz * gz), (gx, gy, gz)


def _face_avg(a, axis, bc_letter):
    """1/2 (a[i] + a[i+1]) on face i+1/2; zero on a wall face, the inner
    cell's value on an outflow face."""
    out = 0.5 * (a + np.roll(a, -1, axis=axis))
    sl = [slice(None)] * 3
    sl[axis] = -1
    if bc_letter == "N":
        out[tuple(sl)] = 0.0
    elif bc_letter == "D":
        out[tuple(sl)] = a[tuple(sl)]
    return out


def interface_normal_faces(C, dx, dy, dzf, bc: str, scale: float):
    """scale * n on faces, n = -grad C / |grad C| at centres (the normal
    pointing out of the phase where C = 1), averaged to faces.

    With scale = mdot / rho1 this is the q term of the interface velocity
    u_G = u_1^e - (mdot / rho1) n (section 3.6).
    """
    bc = _check_bc(bc)
    mag, (gx, gy, gz) = grad_mag_central(C, dx, dy, dzf, bc)
    safe = np.where(mag > 1e-12, mag, 1.0)
    nxc = -np.where(mag > 1e-12, gx / safe, 0.0) * scale
    nyc = -np.where(mag > 1e-12, gy / safe, 0.0) * scale
    nzc = -np.where(mag > 1e-12, gz / safe, 0.0) * scale
    return (_face_avg(nxc, 2, bc[0]), _face_avg(nyc, 1, bc[1]),
            _face_avg(nzc, 0, bc[2]))


# ----------------------------------------------------------------------------
# discretely solenoidal velocity: the MAC curl of a seeded edge potential
# ----------------------------------------------------------------------------
def _back(a, axis, bc_letter):
    """a shifted so that entry i holds a[i-1]; wrap (P) or zero at -1 (N)."""
    if bc_letter == "P":
        return np.roll(a, 1, axis=axis)
    out = np.zeros_like(a)
    sl_dst = [slice(None)] * 3
    sl_src = [slice(None)] * 3
    sl_dst[axis] = slice(1, None)
    sl_src[axis] = slice(None, -1)
    out[tuple(sl_dst)] = a[tuple(sl_src)]
    return out


def solenoidal_faces(nx, ny, nz, dx, dy, dzf, bc: str, seed: int):
    """Face velocity u = curl A of a seeded edge potential A ~ N(0,1).

    A_x lives on edges (i, j+1/2, k+1/2), A_y on (i+1/2, j, k+1/2) and A_z on
    (i+1/2, j+1/2, k).  Edge values lying in a wall plane are zero, so the
    velocity vanishes on wall faces.  Each face value is a difference of
    edge values over the cell width, hence the cell divergence of u cancels
    term by term for any grid widths.
    """
    bc = _check_bc(bc)
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    Ax = rng.standard_normal(size=shape)
    Ay = rng.standard_normal(size=shape)
    Az = rng.standard_normal(size=shape)
    if bc[0] == "N":
        Ay[:, :, -1] = 0.0
        Az[:, :, -1] = 0.0
    if bc[1] == "N":
        Ax[:, -1, :] = 0.0
        Az[:, -1, :] = 0.0
    if bc[2] == "N":
        Ax[-1, :, :] = 0.0
        Ay[-1, :, :] = 0.0
    dz = np.asarray(dzf, dtype=np.float64)[:, None, None]
    u = (Az - _back(Az, 1, bc[1])) / dy - (Ay - _back(Ay, 0, bc[2])) / dz
    v = (Ax - _back(Ax, 0, bc[2])) / dz - (Az - _back(Az, 2, bc[0])) / dx
    w = (Ay - _back(Ay, 2, bc[0])) / dx - (Ax - _back(Ax, 1, bc[1])) / dy
    return _zero_walls(u, v, w, bc)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Config:
    name: str
    nx: int
    ny: int
    nz: int
    bc: str
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    beta: float | None = None  # None: uniform z

    @property
    def dx(self):
        return self.lx / self.nx

    @property
    def dy(self):
        return self.ly / self.ny

    def dzf(self):
        if self.beta is None:
            return uniform_dz(self.nz, self.lz)
        return stretched_dz(self.nz, self.lz, self.beta)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def npts(self):
        return self.nx * self.ny * self.nz


CONFIGS = {
    # 32^3 triply periodic, L = 1
    "ppp32": Config("ppp32", 32, 32, 32, "PPP"),
    # 128^3, periodic x/y, walls in z, uniform
    "ppn128": Config("ppn128", 128, 128, 128, "PPN"),
    # the 256^3 solve the throughput metric is quoted on (periodic x/y, walls z)
    "ppn256": Config("ppn256", 256, 256, 256, "PPN"),
    # 512x512x256, walls in z, tanh clustering beta = 1.5
    "ppn512s": Config("ppn512s", 512, 512, 256, "PPN", beta=1.5),
    # 512^3 triply periodic (mixed-precision comparison)
    "ppp512": Config("ppp512", 512, 512, 512, "PPP"),
    # the three-dimensional settling droplet grid: 320 x 320 x 640 cubic cells,
    # triply periodic (transform lengths 5 * 2^k)
    "ppp320x320x640": Config("ppp320x320x640", 320, 320, 640, "PPP", lz=2.0),
    # serving classes
    "ppn64": Config("ppn64", 64, 64, 64, "PPN"),
    "ppn128x128x256s": Config("ppn128x128x256s", 128, 128, 256, "PPN", beta=1.5),
    "slab1024": Config("slab1024", 1024, 1024, 1, "PPN", lz=1.0 / 1024),
}


def config(name: str) -> Config:
    return CONFIGS[name]
