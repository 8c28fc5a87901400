"""Laser scan path and the heat loads (paper Section 5.2).

Readings:
  * Surface model (the default): a Gaussian flux on the top surface, in the
    paper's exponent convention,
        q(x, y) = 3 eta P / (pi R^2) * exp(-3 ((x-x_c)^2 + (y-y_c)^2) / R^2),
    whose integral over the plane is exactly eta P; the coarse level takes
    the time average of the loads at the m micro times.
  * Volume model (the paper's Section 5.2 sources):
      - local level: the volumetric Gaussian of radius R and depth d
        centred on the spot at the top surface,
            Q-(x, y, z) = A exp(-3 ((x-x_c)^2 + (y-y_c)^2) / R^2
                                - 3 (z - z_top)^2 / d^2),
        with A = 6 sqrt(3) eta P / (pi^(3/2) R^2 d).  The paper prints the
        prefactor with 2 pi in place of pi^(3/2); that version does not
        absorb eta P in the half-space below the surface, so A is taken
        from the normalisation the paper intends (the source carries the
        beam's absorbed power);
      - global level: a constant source eta P / (R d v Dt) in the box the
        beam sweeps during the macro step -- v Dt along the track, R
        across it (centred), d below the top -- so the step receives eta P
        Dt.  A step that ends one track and starts the next gets one box
        per piece, each of length v tau for the time tau spent on it.
        Boxes are axis-aligned, so the volume model takes tracks along x
        or along y.
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


# ---------------------------------------------------------------------------
# volume model
# ---------------------------------------------------------------------------
def volume_amplitude(P, eta, R, d):
    """A of the volumetric Gaussian: eta P over the half-space z < z_top."""
    return 6.0 * np.sqrt(3.0) * eta * P / (np.pi ** 1.5 * R * R * d)


def volume_density(x, y, z, spot, depth, z_top):
    """Q-(x, y, z) in W/m^3 of the spot (depth d, surface at z_top)."""
    xc, yc, P, R, eta = spot[:5]
    A = volume_amplitude(P, eta, R, depth)
    return A * np.exp(-3.0 * ((x - xc) ** 2 + (y - yc) ** 2) / (R * R)
                      - 3.0 * (z - z_top) ** 2 / (depth * depth))


def _gauss_moments(a, b, c, alpha):
    """int_a^b exp(-alpha (x-c)^2) dx and int_a^b x exp(-alpha (x-c)^2) dx."""
    from scipy.special import erf
    sa = np.sqrt(alpha)
    m0 = 0.5 * np.sqrt(np.pi / alpha) * (erf(sa * (b - c)) - erf(sa * (a - c)))
    m1 = c * m0 - (np.exp(-alpha * (b - c) ** 2) - np.exp(-alpha * (a - c) ** 2)) / (2.0 * alpha)
    return m0, m1


def _hat_gauss(n_nodes, x0, h, c, alpha):
    """G_i = int exp(-alpha (x-c)^2) phi_i(x) dx along one axis of a grid with
    nodes x0 + i h (i = 0..n_nodes-1), phi_i the 1D hat functions, by the
    closed forms of _gauss_moments on the cells left and right of each
    node."""
    G = np.zeros(n_nodes)
    xs = x0 + h * np.arange(n_nodes)
    for i in range(n_nodes):
        if i > 0:                       # rising part on [x_{i-1}, x_i]
            m0, m1 = _gauss_moments(xs[i - 1], xs[i], c, alpha)
            G[i] += (m1 - xs[i - 1] * m0) / h
        if i < n_nodes - 1:             # falling part on [x_i, x_{i+1}]
            m0, m1 = _gauss_moments(xs[i], xs[i + 1], c, alpha)
            G[i] += (xs[i + 1] * m0 - m1) / h
    return G


def volume_load(grid, spot, depth, z_top):
    """F_i = int Q- phi_i dV over the whole grid.  Q- and the Q1 basis are
    products of one factor per axis, so F_i = A Gx(i) Gy(j) Gz(k) with the
    1D integrals of _hat_gauss."""
    F = np.zeros(grid.n_nodes)
    if spot is None:
        return F
    xc, yc, P, R, eta = spot[:5]
    A = volume_amplitude(P, eta, R, depth)
    Gx = _hat_gauss(grid.nx + 1, grid.x0, grid.hx, xc, 3.0 / (R * R))
    Gy = _hat_gauss(grid.ny + 1, grid.y0, grid.hy, yc, 3.0 / (R * R))
    Gz = _hat_gauss(grid.nz + 1, grid.z0, grid.hz, z_top, 3.0 / (depth * depth))
    i, j, k = grid.node_ijk()
    return A * Gx[i] * Gy[j] * Gz[k]


def swept_boxes(scan, t0, t1, z_top):
    """The boxes of the global source for the step [t0, t1]: for every piece
    of track the beam covers in it, (x_lo, x_hi, y_lo, y_hi, z_lo, z_hi,
    density) with density eta P / (R d v (t1 - t0))."""
    starts, t_end = track_start_times(scan)
    out = []
    for k, tr in enumerate(scan.tracks):
        length = np.hypot(tr.x1 - tr.x0, tr.y1 - tr.y0)
        ts, te = starts[k], starts[k] + length / tr.speed
        a, b = max(t0, ts), min(t1, te)
        if b <= a:
            continue
        ux, uy = (tr.x1 - tr.x0) / length, (tr.y1 - tr.y0) / length
        pa = (tr.x0 + ux * tr.speed * (a - ts), tr.y0 + uy * tr.speed * (a - ts))
        pb = (tr.x0 + ux * tr.speed * (b - ts), tr.y0 + uy * tr.speed * (b - ts))
        R, d = tr.radius, tr.depth
        if abs(uy) < 1e-12:        # along x
            x_lo, x_hi = min(pa[0], pb[0]), max(pa[0], pb[0])
            y_lo, y_hi = pa[1] - 0.5 * R, pa[1] + 0.5 * R
        else:                      # along y
            x_lo, x_hi = pa[0] - 0.5 * R, pa[0] + 0.5 * R
            y_lo, y_hi = min(pa[1], pb[1]), max(pa[1], pb[1])
        q = tr.absorptivity * tr.power / (R * d * tr.speed * (t1 - t0))
        out.append((x_lo, x_hi, y_lo, y_hi, z_top - d, z_top, q))
    return out


def _hat_box(lo, hi, e0, h):
    """int over [lo, hi] ∩ [e0, e0 + h] of the two 1D basis functions of the
    cell [e0, e0 + h]: (falling, rising)."""
    a = np.clip(lo, e0, e0 + h)
    b = np.clip(hi, e0, e0 + h)
    rise = ((b - e0) ** 2 - (a - e0) ** 2) / (2.0 * h)
    return (b - a) - rise, rise


def box_load(grid, boxes, elem_mask=None):
    """F_i = sum over boxes of q int_{box ∩ elements} phi_i dV, exact: the part
    of an element inside an axis-aligned box is a box, and the integral of
    a trilinear basis function over it is a product of 1D integrals
    (_hat_box).  elem_mask keeps only the elements where it is nonzero."""
    F = np.zeros(grid.n_nodes)
    ei, ej, ek = grid.elem_ijk()
    keep = np.ones(grid.n_elems, bool) if elem_mask is None else np.asarray(elem_mask) != 0
    corners = grid.element_corners()
    for (x_lo, x_hi, y_lo, y_hi, z_lo, z_hi, q) in boxes:
        fx = _hat_box(x_lo, x_hi, grid.x0 + ei * grid.hx, grid.hx)
        fy = _hat_box(y_lo, y_hi, grid.y0 + ej * grid.hy, grid.hy)
        fz = _hat_box(z_lo, z_hi, grid.z0 + ek * grid.hz, grid.hz)
        for c in range(8):
            a, b, g = c & 1, (c >> 1) & 1, c >> 2
            val = q * fx[a] * fy[b] * fz[g]
            np.add.at(F, corners[keep, c], val[keep])
    return F
