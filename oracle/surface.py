"""Heat loss through the top surface z = top (paper Section 2, boundary
conditions of the thermal problem).

The paper's local problem loses heat through its upper surface by
convection and radiation, q(T) = h (T - T_amb) + sigma eps (T^4 - T_amb^4);
its global problem by convection only, q(T) = h (T - T_amb) (radiation is
neglected away from the heat-affected zone, which lies in the local
window).  The flux leaves the body, so it enters the residual of a level as

    R_i += A_i q(T_i),     dR_i/dT_i = A_i q'(T_i),

with A_i the lumped area of the top faces around node i (each face gives a
quarter of its area to each corner) -- the surface counterpart of the
lumped nodal mass.  The derivative is exact and positive, so the Jacobian
stays symmetric positive definite.

The Stefan-Boltzmann constant is the physical 5.670374419e-8 W/m^2/K^4; the
paper prints 5.87e-8, read here as a typographical slip.

Test infrastructure: this module is the oracle's, not the product's.
"""
import numpy as np

SIGMA_SB = 5.670374419e-8


def top_area(grid, face_mask=None):
    """Lumped nodal area of the top faces of `grid` (nodes off the top
    layer get 0).  face_mask, over the nx*ny top faces in x-fastest order,
    keeps only the faces where it is true."""
    A = np.zeros(grid.n_nodes)
    fj, fi = np.meshgrid(np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
    fi, fj = fi.ravel(), fj.ravel()
    keep = np.ones(fi.size, dtype=bool) if face_mask is None else np.asarray(face_mask, bool)
    quarter = 0.25 * grid.hx * grid.hy
    for a in (0, 1):
        for b in (0, 1):
            np.add.at(A, grid.node(fi[keep] + a, fj[keep] + b, grid.nz), quarter)
    return A


def flux(T, h, eps, T_amb):
    """Outward heat flux density [W/m^2] at surface temperature T."""
    return h * (T - T_amb) + SIGMA_SB * eps * (T ** 4 - T_amb ** 4)


def flux_slope(T, h, eps, T_amb):
    return h + 4.0 * SIGMA_SB * eps * T ** 3


class Surface:
    """Top-surface loss of one level: nodal areas and the law's parameters."""

    def __init__(self, area, h, eps, T_amb):
        self.area = np.asarray(area, dtype=np.float64)
        self.h, self.eps, self.T_amb = float(h), float(eps), float(T_amb)

    @property
    def active(self):
        return self.h != 0.0 or self.eps != 0.0

    def term(self, T):
        return self.area * flux(T, self.h, self.eps, self.T_amb)

    def slope(self, T):
        return self.area * flux_slope(T, self.h, self.eps, self.T_amb)

    def loss(self, T):
        """Total outward heat flow [W]."""
        return float(np.sum(self.term(T)))
