"""Interface terms from the volume fraction C (test oracle, FP64).

Section 3.2 regularises the interface delta as |grad C| and section 3.4 takes
the normal from grad C / |grad C|, both with the gradient of C evaluated by
Youngs' finite differences; section 3.6 then needs the Stefan source
s = mdot (1/rho2 - 1/rho1) |grad C| at cell centres and the interface-velocity
jump q = (mdot / rho1) n on the velocity faces.

Orientation of n.  The jump condition of section 2 (eq. rankine) defines n as
pointing into phase 2, and the interface velocity of section 3.6 (eq.
int_vel) is derived from it; C is 1 in phase 1 (eq. ind_fun), so grad C points
into phase 1.  Section 3.4 writes n = grad C / |grad C| for the mass-flux
formula; taken literally that orientation would make u_Gamma = u_1^e - q move
an evaporating interface (mdot > 0) into the gas.  The reading taken here is
the one eq. int_vel needs: n = -grad C / |grad C| (into phase 2), so that an
evaporating droplet's interface recedes into the liquid at mdot / rho1.  For boiling (appendix A) the
interface velocity is built from the divergence-free extension of the vapour
velocity instead of the liquid's.  The reading: the potential and the
extension u - grad phi are the same (it follows whichever phase lies where the
potential is harmonic and constant, e.g. inside a closed bubble), and the jump
becomes q = (mdot / rho2) n (phase = 2).

The paper does not print the stencil of the gradient; the reading taken here
is Youngs' corner construction:

1. ghost cells beyond the domain: periodic copies, or mirrored values
   (C and mdot continued with zero normal gradient) at walls and outflow
   ends;
2. the gradient at every cell corner (i+1/2, j+1/2, k+1/2) from the eight
   cells around it: each component is the mean of the four differences across
   the corner along that axis, divided by the centre distance (dx, dy, or dzc
   of the face k+1/2; the mirrored ghost's distance is irrelevant, its
   difference is zero);
3. the gradient at a cell centre as the mean of its eight corner gradients.
On a uniform grid this is the central difference of C weighted (1, 2, 1) in
each transverse direction.  Then |grad C|, n = -grad C / |grad C| (0 where
|grad C| = 0),
s = mdot (1/rho2 - 1/rho1) |grad C| and the cell vector a = (mdot / rho) n
(rho of the extended phase);
q on face i+1/2 is the mean of a at cells i and i+1, and 0 on a non-periodic
boundary face (the mirrored ghost carries the opposite normal component).
"""
from __future__ import annotations

import numpy as np


def _pad(f, g):
    """f with one ghost layer on every side: wrapped (periodic) or mirrored."""
    out = np.asarray(f, dtype=np.float64)
    for axis, (lo, _) in ((2, g.ends[0]), (1, g.ends[1]), (0, g.ends[2])):
        widths = [(0, 0)] * 3
        widths[axis] = (1, 1)
        out = np.pad(out, widths, mode="wrap" if lo == "P" else "edge")
    return out


def _z_centre_distances(g):
    """Distance across each of the nz+1 faces -1/2 .. nz-1/2 between the
    (possibly ghost) cells on either side; ghost widths copy the end cells
    (periodic: the wrapped cell)."""
    dzf = g.dzf
    if g.ends[2][0] == "P":
        ext = np.concatenate([[dzf[-1]], dzf, [dzf[0]]])
    else:
        ext = np.concatenate([[dzf[0]], dzf, [dzf[-1]]])
    return 0.5 * (ext[:-1] + ext[1:])


def corner_gradients(C, g):
    """(gx, gy, gz) at the (nz+1, ny+1, nx+1) corners; corner (k, j, i) sits
    at (i-1/2, j-1/2, k-1/2)."""
    P = _pad(C, g)  # (nz+2, ny+2, nx+2); P[k+1, j+1, i+1] = C[k, j, i]
    dzc = _z_centre_distances(g)  # distance across face k-1/2, k = 0..nz
    # the eight cells around corner (k, j, i) are P[k + a, j + b, i + c], a, b, c in {0, 1}
    def cell(a, b, c):
        return P[a:a + g.nz + 1, b:b + g.ny + 1, c:c + g.nx + 1]
    gx = sum(cell(a, b, 1) - cell(a, b, 0) for a in (0, 1) for b in (0, 1)) / (4.0 * g.dx)
    gy = sum(cell(a, 1, c) - cell(a, 0, c) for a in (0, 1) for c in (0, 1)) / (4.0 * g.dy)
    gz = sum(cell(1, b, c) - cell(0, b, c) for b in (0, 1) for c in (0, 1)) / (
        4.0 * dzc[:, None, None])
    return gx, gy, gz


def youngs_gradient(C, g):
    """grad C at the cell centres: the mean of the eight corner gradients."""
    out = []
    for comp in corner_gradients(C, g):
        acc = 0.0
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    acc = acc + comp[a:a + g.nz, b:b + g.ny, c:c + g.nx]
        out.append(acc / 8.0)
    return tuple(out)


def interface_terms(C, mdot, rho1, rho2, g, phase=1):
    """(s, qx, qy, qz, |grad C|) as described in the module docstring; `phase`
    is the phase whose velocity the extension follows (1 liquid, 2 vapour)."""
    if phase not in (1, 2):
        raise ValueError("phase must be 1 (liquid) or 2 (vapour)")
    gx, gy, gz = youngs_gradient(C, g)
    mag = np.sqrt(gx * gx + gy * gy + gz * gz)
    mdot = np.asarray(mdot, dtype=np.float64)
    s = mdot * (1.0 / rho2 - 1.0 / rho1) * mag
    safe = np.where(mag > 0.0, mag, 1.0)
    rho_ext = rho1 if phase == 1 else rho2
    # n = -grad C / |grad C|: into phase 2 (see the module docstring)
    scale = np.where(mag > 0.0, -mdot / rho_ext / safe, 0.0)
    q = []
    for axis, comp in ((2, gx), (1, gy), (0, gz)):
        a = scale * comp
        face = 0.5 * (a + np.roll(a, -1, axis=axis))
        if g.ends[2 - axis][0] != "P":
            sl = [slice(None)] * 3
            sl[axis] = -1
            face[tuple(sl)] = 0.0
        q.append(face)
    return s, q[0], q[1], q[2], mag
