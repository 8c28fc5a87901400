"""Laser scan path and the surface heat load (paper Section 5.2).

Readings:
  * The paper uses a volumetric Gaussian in the local problem and a smeared
    box source in the global one (Section 5.2).  Here the laser is a
    Gaussian flux on the top surface, in the paper's exponent convention:
        q(x, y) = 3 eta P / (pi R^2) * exp(-3 ((x-x_c)^2 + (y-y_c)^2) / R^2),
    whose integral over the plane is exactly eta P.
  * The beam moves along straight tracks at constant speed, one after the
    other with no jump time, starting at t_start; it is off before the
    first track starts and after the last one ends.
  * The load vector is F_i = sum over top faces of int q phi_i dA, each face
    integrated with n_q x n_q Gauss-Legendre points.
"""
import numpy as np


def track_start_times(scan):
    """Start time of every track and the end time of the last one."""
    starts = []
    t = scan.t_start
    for tr in scan.tracks:
        starts.append(t)
        length = np.hypot(tr.x1 - tr.x0, tr.y1 - tr.y0)
        t = t + length / tr.speed
    return starts, t


def laser_at(scan, t):
    """Spot state at time t: (x_c, y_c, power, radius, absorptivity, k) for
    track k, or None when the beam is off."""
    starts, t_end = track_start_times(scan)
    if t < scan.t_start or t > t_end or not scan.tracks:
        return None
    k = len(starts) - 1
    for q in range(len(starts) - 1):
        if t < starts[q + 1]:
            k = q
            break
    tr = scan.tracks[k]
    length = np.hypot(tr.x1 - tr.x0, tr.y1 - tr.y0)
    s = (t - starts[k]) * tr.speed
    frac = s / length if length > 0 else 0.0
    if frac > 1.0:
        frac = 1.0
    xc = tr.x0 + (tr.x1 - tr.x0) * frac
    yc = tr.y0 + (tr.y1 - tr.y0) * frac
    return (xc, yc, tr.power, tr.radius, tr.absorptivity, k)


def surface_flux(x, y, spot):
    """Absorbed flux density q(x, y) in W/m^2 of the spot."""
    xc, yc, P, R, eta = spot[:5]
    return 3.0 * eta * P / (np.pi * R * R) * np.exp(-3.0 * ((x - xc) ** 2 + (y - yc) ** 2) / (R * R))


def gauss01(nq):
    """Gauss-Legendre points and weights mapped to [0, 1]."""
    p, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (p + 1.0), 0.5 * w


def top_load(grid, spot, nq=3, face_mask=None):
    """F_i = sum_faces int_face q phi_i dA over the top faces z = z0 + nz hz.
    face_mask (nx*ny booleans, face (i, j) at i + nx j) restricts the faces.
    Returns a vector over all nodes of the grid."""
    F = np.zeros(grid.n_nodes)
    if spot is None:
        return F
    xi, wq = gauss01(nq)
    fj, fi = np.meshgrid(np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
    fi, fj = fi.ravel(), fj.ravel()
    if face_mask is not None:
        keep = np.asarray(face_mask, dtype=bool)
        fi, fj = fi[keep], fj[keep]
    k = grid.nz
    area = grid.hx * grid.hy
    for qa in range(nq):
        for qb in range(nq):
            x = grid.x0 + (fi + xi[qa]) * grid.hx
            y = grid.y0 + (fj + xi[qb]) * grid.hy
            qv = surface_flux(x, y, spot) * (wq[qa] * wq[qb] * area)
            for b in (0, 1):
                for a in (0, 1):
                    phi = (xi[qa] if a else 1.0 - xi[qa]) * (xi[qb] if b else 1.0 - xi[qb])
                    np.add.at(F, grid.node(fi + a, fj + b, k), qv * phi)
    return F
