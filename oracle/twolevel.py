"""The spatiotemporal two-level method (paper Sections 3 and 4, Algorithm 1).

Global (coarse) temperature T+ lives on the whole plate Omega+; local (fine)
temperature T- lives on a window Omega- that follows the laser (Section 5.2
moves the local mesh with the beam).  Within macro step t_n -> t_n + Dt:

  1. place the window (rule below); on a move, copy the overlap of the old
     fine field and fill newly covered fine nodes by trilinear interpolation
     P of the coarse field (the paper moves the local mesh without any other
     projection, Section 5.2);
  2. predictor: one coarse implicit step over all elements with the load
     averaged over the macro step, giving the intermediate T~+ (Algorithm 1);
  3. micro steps j = 1..m-1: fine implicit steps of size dt = Dt/m whose
     Dirichlet data on the immersed window boundary gamma_D blend the two
     coarse fields, (1 - j/m) P T+^n + (j/m) P T~+ (the time-local problem of
     Section 4);
  4. correction at t_n + Dt: the two-level iteration of Section 3, solved
     "possibly relaxed, until convergence".

Readings adopted where the paper is silent, ambiguous or garbled:
  * Indexing of Algorithm 1: its loop "i = 0..m-1 at t_n + i dt" is read as
    implicit steps landing at t_n + j dt, j = 1..m-1, with boundary data at
    the new time level; step j = m is the coupled correction.  With m = 1
    there are no intermediate steps.
  * Discrete two-level iteration: Dirichlet-Neumann.  The local problem takes
    T- = T+ on gamma_D (Section 3, zero temperature jump); the global problem
    is solved on the elements outside the window, with the coarse nodes
    strictly inside the window fixed to the local solution and the local
    side's reaction flux entering the coarse interface rows through the
    transpose of P -- the discrete form of the interface functional xi_gamma
    and of the zero flux jump (Section 3).  Both levels use the same material
    law, so the alternate formulation's jump term (kappa+ - kappa-) vanishes;
    this reading keeps the paper's statement that equal global and local
    steps reproduce the single-level solution (Section 5.1).
  * The interface load averages the reactions of all m micro steps (not only
    the last), which makes the energy ledger exact for every m.
  * Relaxation lambda <- lambda + theta (lambda' - lambda), with either a
    fixed theta or (default) Aitken's delta-squared rule started from
    r/(r+1); stopped when max |lambda' - lambda| <= dn_tol.  Any relaxation
    converges to the same fixed point.
  * Latent heat is kept on both levels (one material law).
  * Window rule: whole coarse cells, flush with the top, centred on the beam
    across the scan direction; along it the beam position at t_{n+1} sits one
    third of the window length behind the leading edge; clamped inside the
    plate; kept in place while the beam is off.
  * Coarse load: the time average of the surface loads at the m micro times
    (the intent of the paper's smeared global source, Section 5.2); with the
    volume model, the paper's sources themselves (oracle.laser).
  * Top-surface heat loss (Section 2): convection and radiation on the fine
    level's top faces, convection only on the coarse level's (the window's
    faces excluded in the outside solve); lumped over the faces' corners
    (oracle.surface).  The ledger then reads
    E_{n+1} - E_n = absorbed - bottom - surface + remap.
"""
import math
from dataclasses import replace

import numpy as np
import scipy.sparse as sp

from . import grid as G
from . import laser as L
from . import material as M
from . import surface as S
from .level import (implicit_step, residual, solve_spd, NoConvergence, LINE_SEARCH_MAX,
                    Fictitious)


class Window:
    """Geometry of one window position: fine grid, node classes, transfers."""

    def __init__(self, coarse, mesh, I0, J0):
        r = mesh.refine
        self.I0, self.J0 = I0, J0
        self.K0 = mesh.nz - mesh.win_nz
        self.wx, self.wy, self.wz = mesh.win_nx, mesh.win_ny, mesh.win_nz
        c = coarse
        self.fine = G.Grid(r * self.wx, r * self.wy, r * self.wz,
                           c.hx / r, c.hy / r, c.hz / r,
                           I0 * c.hx, J0 * c.hy, self.K0 * c.hz)
        f = self.fine
        # which window faces are immersed (not on the plate boundary)
        self.face_x0 = I0 > 0
        self.face_x1 = I0 + self.wx < mesh.nx
        self.face_y0 = J0 > 0
        self.face_y1 = J0 + self.wy < mesh.ny
        self.face_z0 = self.K0 > 0
        # fine node classes
        fi, fj, fk = f.node_ijk()
        # a window reaching the plate bottom has its bottom row fixed at
        # T_bottom; such nodes count as bottom, not as interface, nodes
        self.bottom_f = (fk == 0) & (self.K0 == 0)
        self.gamma_f = ((self.face_x0 & (fi == 0)) | (self.face_x1 & (fi == f.nx))
                        | (self.face_y0 & (fj == 0)) | (self.face_y1 & (fj == f.ny))
                        | (self.face_z0 & (fk == 0))) & ~self.bottom_f
        self.dir_f = self.gamma_f | self.bottom_f
        # coarse node classes
        ci, cj, ck = c.node_ijk()
        inwin = ((ci >= I0) & (ci <= I0 + self.wx) & (cj >= J0) & (cj <= J0 + self.wy)
                 & (ck >= self.K0))
        on_gamma = ((self.face_x0 & (ci == I0)) | (self.face_x1 & (ci == I0 + self.wx))
                    | (self.face_y0 & (cj == J0)) | (self.face_y1 & (cj == J0 + self.wy))
                    | (self.face_z0 & (ck == self.K0)))
        self.gamma_c = inwin & on_gamma
        self.interior_c = inwin & ~on_gamma
        # coarse elements outside the window, coarse top faces outside it
        ei, ej, ek = c.elem_ijk()
        e_in = ((ei >= I0) & (ei < I0 + self.wx) & (ej >= J0) & (ej < J0 + self.wy)
                & (ek >= self.K0))
        self.outside_e = (~e_in).astype(np.float64)
        fj2, fi2 = np.meshgrid(np.arange(c.ny), np.arange(c.nx), indexing="ij")
        fi2, fj2 = fi2.ravel(), fj2.ravel()
        self.outside_face = ~((fi2 >= I0) & (fi2 < I0 + self.wx)
                              & (fj2 >= J0) & (fj2 < J0 + self.wy))
        self.mass_out = G.lumped_mass(c, self.outside_e)
        self.mass_in = G.lumped_mass(c, 1.0 - self.outside_e)
        self.mass_f = G.lumped_mass(f)
        # lumped top-surface areas: every fine top face; coarse top faces
        # outside the window
        self.area_f = S.top_area(f)
        self.area_out = S.top_area(c, self.outside_face)
        # injection: coarse window-interior node -> fine node at its position
        idx = np.flatnonzero(self.interior_c)
        self.inject_c = idx
        self.inject_f = f.node(r * (ci[idx] - I0), r * (cj[idx] - J0), r * (ck[idx] - self.K0))
        self.P = prolongation(c, f, r, I0, J0, self.K0)


def prolongation(coarse, fine, r, I0, J0, K0):
    """Trilinear interpolation P from coarse nodes to the fine nodes of a
    window whose fine grid starts at coarse node (I0, J0, K0); n_fine x
    n_coarse sparse matrix."""
    fi, fj, fk = fine.node_ijk()
    axes = []
    for loc, start, ncell in ((fi, I0, coarse.nx), (fj, J0, coarse.ny), (fk, K0, coarse.nz)):
        g = r * start + loc                      # global fine index on this axis
        cell = np.minimum(g // r, ncell - 1)     # coarse cell containing it
        frac = (g - cell * r) / r                # position inside that cell
        axes.append((cell, frac))
    rows, cols, vals = [], [], []
    for g_ in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                (cx, fx), (cy, fy), (cz, fz) = axes
                w = ((fx if a else 1.0 - fx) * (fy if b else 1.0 - fy)) * (fz if g_ else 1.0 - fz)
                rows.append(np.arange(fine.n_nodes))
                cols.append(coarse.node(cx + a, cy + b, cz + g_))
                vals.append(w)
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.n_nodes, coarse.n_nodes))
    return P


def window_origin(mesh, coarse, scan, t, current=None):
    """Window position (I0, J0) in coarse cells for beam time t (rule in the
    module docstring).  Returns `current` when the beam is off."""
    spot = L.laser_at(scan, t)
    if spot is None:
        if current is not None:
            return current
        tr = scan.tracks[0]
        spot = (tr.x0, tr.y0, tr.power, tr.radius, tr.absorptivity, 0)
    xc, yc, k = spot[0], spot[1], spot[5]
    tr = scan.tracks[k]
    dx, dy = tr.x1 - tr.x0, tr.y1 - tr.y0
    wx_len = mesh.win_nx * coarse.hx
    wy_len = mesh.win_ny * coarse.hy
    if abs(dx) >= abs(dy):
        lead = (2.0 / 3.0) if dx >= 0 else (1.0 / 3.0)
        x_lo = xc - lead * wx_len
        y_lo = yc - 0.5 * wy_len
    else:
        lead = (2.0 / 3.0) if dy >= 0 else (1.0 / 3.0)
        x_lo = xc - 0.5 * wx_len
        y_lo = yc - lead * wy_len
    I0 = int(math.floor(x_lo / coarse.hx + 0.5))
    J0 = int(math.floor(y_lo / coarse.hy + 0.5))
    I0 = min(max(I0, 0), mesh.nx - mesh.win_nx)
    J0 = min(max(J0, 0), mesh.ny - mesh.win_ny)
    return (I0, J0)


def coarse_grid(mesh):
    return G.Grid(mesh.nx, mesh.ny, mesh.nz, mesh.lx / mesh.nx, mesh.ly / mesh.ny,
                  mesh.lz / mesh.nz)


def micro_time(scan, opts, n, j):
    """Time of micro step j (0..m) of macro step n."""
    return scan.t_start + n * opts.dt_coarse + j * (opts.dt_coarse / opts.m_time)


class TwoLevel:
    """State and macro step of the spatiotemporal two-level method."""

    def __init__(self, wl, newton_tol=None, dn_tol=None, composite=False):
        """The correction runs the Dirichlet-Neumann iteration of Section 3
        unless `composite` asks for the composite-grid solve of the same
        equations (composite_correction); the workload's own choice of
        solver for the GPU path does not change the oracle."""
        self.wl = wl
        self.composite = bool(composite)
        # the alternate global formulation is a different discrete problem,
        # so the oracle follows the workload there
        self.alternate = getattr(wl.options, "coupling", 0) == 2
        # the consistent global formulation (Section 3) with constant global
        # coefficients inside the window: another discrete problem too
        self.consistent = getattr(wl.options, "coupling", 0) == 3
        self.volume = getattr(wl.options, "source", 0) == 1
        self.z_top = wl.mesh.lz
        mesh, mat, opts = wl.mesh, wl.material, wl.options
        if mesh.win_nx > mesh.nx or mesh.win_ny > mesh.ny or mesh.win_nz > mesh.nz:
            raise ValueError("window larger than the plate")
        self.mesh, self.mat, self.scan, self.opts = mesh, mat, wl.scan, opts
        self.newton_tol = opts.newton_tol if newton_tol is None else newton_tol
        self.dn_tol = opts.dn_tol if dn_tol is None else dn_tol
        r = mesh.refine
        self.fixed_theta = opts.dn_theta > 0
        self.theta = opts.dn_theta if self.fixed_theta else r / (r + 1.0)
        self.coarse = coarse_grid(mesh)
        c = self.coarse
        _, _, ck = c.node_ijk()
        self.bottom_c = ck == 0
        self.Tc = np.full(c.n_nodes, mat.T_init)
        self.Tc[self.bottom_c] = mat.T_bottom
        self.n = 0
        origin = window_origin(mesh, c, self.scan, micro_time(self.scan, opts, 1, 0))
        self.win = Window(c, mesh, *origin)
        self.Tf = np.full(self.win.fine.n_nodes, mat.T_init)
        self.Tf[self.win.bottom_f] = mat.T_bottom
        self.area_c = S.top_area(c)
        # the alternate formulation's global problem: all elements, the same
        # law without latent heat (the paper keeps latent heat in the local
        # problem only)
        self.mat_global = replace(mat, latent=0.0) if self.alternate else mat
        self.mass_all = G.lumped_mass(c)
        # the consistent formulation's global coefficients inside the window;
        # zero selects the material law's values at T_init
        T0 = np.array([mat.T_init])
        kf, cf = getattr(mat, "k_fict", 0.0), getattr(mat, "rhoc_fict", 0.0)
        self.k_fict = kf if kf > 0 else float(M.conductivity(T0, mat)[0])
        self.rhoc_fict = cf if cf > 0 else mat.rho * float(M.heat_capacity(T0, mat)[0])
        self.ledger = dict(stored=self.energy(), absorbed=0.0, bottom=0.0, remap=0.0,
                           surface=0.0, stored0=0.0)
        self.ledger["stored0"] = self.ledger["stored"]
        self.stats = dict(newton_fine=0, newton_coarse=0, dn_iters=0, moves=0,
                          fine_solves=0, coarse_solves=0)
        self.history = []
        # (macro step, micro step j, fine field) of every fine step when a
        # list is set here: micro steps j = 1..m-1 and the corrected step m
        self.record = None

    # -- energy ledger ------------------------------------------------------
    def energy(self):
        """E = sum_J m_J^out H(T+_J) + sum_k m_k H(T-_k); with the alternate
        formulation the global problem's own energy, sum_J m_J H+(T+_J)."""
        if self.alternate:
            return float(np.dot(self.mass_all, M.enthalpy(self.Tc, self.mat_global)))
        w = self.win
        if self.consistent:
            # plus the energy the global problem's own coefficients hold
            # inside the window beyond the local field's (see
            # _correct_consistent)
            return float(np.dot(w.mass_out, M.enthalpy(self.Tc, self.mat))
                         + np.dot(w.mass_f, M.enthalpy(self.Tf, self.mat))
                         + self.rhoc_fict * (np.dot(w.mass_in, self.Tc)
                                             - np.dot(w.mass_f, self.Tf)))
        return float(np.dot(w.mass_out, M.enthalpy(self.Tc, self.mat))
                     + np.dot(w.mass_f, M.enthalpy(self.Tf, self.mat)))

    # -- window move --------------------------------------------------------
    def move_window(self, origin):
        old, mesh = self.win, self.mesh
        new = Window(self.coarse, mesh, *origin)
        r = mesh.refine
        f = new.fine
        fi, fj, fk = f.node_ijk()
        oi = fi + r * (new.I0 - old.I0)
        oj = fj + r * (new.J0 - old.J0)
        inside_old = (oi >= 0) & (oi <= old.fine.nx) & (oj >= 0) & (oj <= old.fine.ny)
        Tnew = new.P @ self.Tc
        Tnew[inside_old] = self.Tf[old.fine.node(oi[inside_old], oj[inside_old], fk[inside_old])]
        self.win = new
        self.Tf = Tnew
        self.stats["moves"] += 1

    def relaxation(self, it, d, d_prev, theta):
        """Relaxation factor of interface update `it` (1-based) given the
        interface residual d = lambda' - lambda and the previous one.  Fixed
        theta when dn_theta > 0, else Aitken's delta-squared rule
            theta_k = -theta_{k-1} <d_{k-1}, d_k - d_{k-1}> / |d_k - d_{k-1}|^2
        started from r/(r+1)."""
        if self.fixed_theta or it == 1:
            return theta
        dd = d - d_prev
        den = float(dd @ dd)
        if den <= 0.0:
            return theta
        return -theta * float(d_prev @ dd) / den

    # -- top-surface loss of each level --------------------------------------
    def surf_fine(self):
        m = self.mat
        return S.Surface(self.win.area_f, m.h_conv, m.emissivity, m.T_amb)

    def surf_coarse(self, area):
        m = self.mat
        return S.Surface(area, m.h_conv, 0.0, m.T_amb)

    # -- laser loads ---------------------------------------------------------
    def fine_load(self, spot):
        """Load of the window at one micro time: the surface Gaussian, or the
        volumetric Gaussian of the volume model (oracle.laser)."""
        if self.volume:
            depth = self.scan.tracks[spot[5]].depth if spot is not None else 1.0
            return L.volume_load(self.win.fine, spot, depth, self.z_top)
        return L.top_load(self.win.fine, spot, self.opts.face_quad)

    # -- one macro step (Algorithm 1) ----------------------------------------
    def fine_step(self, T_prev, tau, load, g, guess=None):
        w = self.win
        vals = np.where(w.bottom_f, self.mat.T_bottom, g)
        T, R, it = implicit_step(w.fine, self.mat, T_prev, tau, load, None, w.dir_f, vals,
                                 T_guess=guess, tol=self.newton_tol, maxit=self.opts.newton_max,
                                 surface=self.surf_fine())
        self.stats["newton_fine"] += it
        self.stats["fine_solves"] += 1
        return T, R

    def step(self):
        mesh, opts, scan, mat = self.mesh, self.opts, self.scan, self.mat
        n, m, Dt = self.n, opts.m_time, opts.dt_coarse
        dt = Dt / m
        c = self.coarse
        origin = window_origin(mesh, c, scan, micro_time(scan, opts, n + 1, 0),
                               current=(self.win.I0, self.win.J0))
        if origin != (self.win.I0, self.win.J0):
            e0 = self.energy()
            self.move_window(origin)
            self.ledger["remap"] += self.energy() - e0
        w = self.win
        E_start = self.energy()
        spots = [L.laser_at(scan, micro_time(scan, opts, n, j)) for j in range(1, m + 1)]
        if self.volume:
            boxes = L.swept_boxes(scan, micro_time(scan, opts, n, 0),
                                  micro_time(scan, opts, n, m), self.z_top)
            Fc_all = L.box_load(c, boxes)
            Fc_out = L.box_load(c, boxes, w.outside_e)
        else:
            Fc_all = sum(L.top_load(c, s, opts.face_quad) for s in spots) / m
            Fc_out = sum(L.top_load(c, s, opts.face_quad, w.outside_face) for s in spots) / m
        if self.alternate:
            return self._step_alternate(spots, Fc_all, E_start)
        # predictor over the whole plate
        Tpred, _, it = implicit_step(c, mat, self.Tc, Dt, Fc_all, None, self.bottom_c,
                                     np.full(c.n_nodes, mat.T_bottom), tol=self.newton_tol,
                                     maxit=opts.newton_max, surface=self.surf_coarse(self.area_c))
        self.stats["newton_coarse"] += it
        self.stats["coarse_solves"] += 1
        PTn = w.P @ self.Tc
        PTp = w.P @ Tpred
        T_prev = self.Tf
        T_start = self.Tf
        T_sum = np.zeros(w.fine.n_nodes)
        rho_sum = np.zeros(w.fine.n_nodes)
        absorbed = 0.0
        bottom = 0.0
        surface = 0.0
        sf = self.surf_fine()
        for j in range(1, m):
            g = (1.0 - j / m) * PTn + (j / m) * PTp
            Ff = self.fine_load(spots[j - 1])
            T_prev, R = self.fine_step(T_prev, dt, Ff, g)
            if self.record is not None:
                self.record.append((n, j, T_prev.copy()))
            rho_sum[w.gamma_f] += R[w.gamma_f]
            T_sum += T_prev
            bottom -= dt * R[w.bottom_f].sum()
            absorbed += dt * Ff.sum()
            surface += dt * sf.loss(T_prev)
        # two-level correction at t_{n+1}
        Ff = self.fine_load(spots[m - 1])
        if self.consistent:
            return self._correct_consistent(T_start, T_prev, T_sum, rho_sum, Ff, Fc_out,
                                            Tpred, absorbed, bottom, surface, E_start)
        if self.composite:
            Tf_m, R_m, Tc_new, Rc, it = self.composite_correction(
                T_prev, dt, Ff, rho_sum, Fc_out, T_prev, Tpred)
            return self._finish(Tf_m, R_m, Tc_new, Rc, it, Ff, Fc_out, absorbed,
                                bottom, surface, E_start)
        lam = Tpred.copy()
        dir_c = self.bottom_c | w.interior_c
        guess_f, guess_c = T_prev, Tpred
        d_prev, theta = None, self.theta
        for it in range(1, opts.dn_max + 1):
            Tf_m, R_m = self.fine_step(T_prev, dt, Ff, w.P @ lam, guess_f)
            rho = np.where(w.gamma_f, rho_sum + R_m, 0.0)
            ext = -(w.P.T @ rho) / m
            vals = np.full(c.n_nodes, mat.T_bottom)
            vals[w.inject_c] = Tf_m[w.inject_f]
            Tc_new, Rc, itc = implicit_step(c, mat, self.Tc, Dt, Fc_out + ext, w.outside_e,
                                            dir_c, vals, T_guess=guess_c, tol=self.newton_tol,
                                            maxit=opts.newton_max,
                                            surface=self.surf_coarse(w.area_out))
            self.stats["newton_coarse"] += itc
            self.stats["coarse_solves"] += 1
            d = np.where(w.gamma_c, Tc_new - lam, 0.0)
            diff = float(np.max(np.abs(d)))
            theta = self.relaxation(it, d, d_prev, theta)
            d_prev = d
            lam = lam + theta * d
            guess_f, guess_c = Tf_m, Tc_new
            if diff <= self.dn_tol:
                break
        else:
            raise NoConvergence("two-level iteration did not converge")
        self._finish(Tf_m, R_m, Tc_new, Rc, it, Ff, Fc_out, absorbed, bottom, surface,
                     E_start)

    def _correct_consistent(self, T_start, T_prev, T_sum, rho_sum, Ff, Fc_out, Tpred,
                            absorbed, bottom, surface, E_start):
        """The two-level correction with the consistent global problem of
        Section 3.  The global problem is posed on every coarse element:
        outside the window with the material law, inside it with the global
        problem's own constant coefficients (k_fict, rhoc_fict), loaded inside
        by the local solution.  Section 3 writes that load as the volume
        terms (the T- time derivative weighted by the coefficient ratios, Q
        scaled by kappa+/kappa-, the two grad T- . grad kappa terms) and the
        interface jump term.  Integrating them against a coarse test function
        and using the local equation, they add up to the global operator with
        the global coefficients applied to T- over the window, minus the
        flux of T- through gamma_D.  Discretely, with the coarse basis in the
        fine space (phi_J = sum_k P_kJ phi_k), that is the load P^T s with
            s = rhoc_fict m_k (T-_m - T-_0) / Dt + k_fict (K1 Tavg)_k - rho_k,
        K1 the unit-conductivity fine stiffness of the window, Tavg the mean
        of the m micro-step fields, rho the mean over the micro steps of the
        local reactions on gamma_D (the local residual, zero on the free rows
        once solved).  The mean over the micro steps is the local equation
        summed over the macro step, so the time term telescopes to the
        change over Dt.  Dirichlet data of the local problem come from T+ on
        gamma_D as before; the iteration between the last micro step and the
        global solve is the same relaxed fixed point on the interface values
        as the Dirichlet-Neumann correction.  The global field keeps its own
        values inside the window (no injection): with equal levels (r = 1,
        m = 1) it equals the local field there and the single-level solution
        everywhere, the stronger consistency of Section 3."""
        mesh, opts, mat, c, w = self.mesh, self.opts, self.mat, self.coarse, self.win
        m, Dt = opts.m_time, opts.dt_coarse
        dt = Dt / m
        fict = Fictitious(c, 1.0 - w.outside_e, self.k_fict, self.rhoc_fict)
        K1 = G.stiffness(w.fine, np.ones(w.fine.n_elems))
        lam = Tpred.copy()
        guess_f, guess_c = T_prev, Tpred
        d_prev, theta = None, self.theta
        for it in range(1, opts.dn_max + 1):
            Tf_m, R_m = self.fine_step(T_prev, dt, Ff, w.P @ lam, guess_f)
            rho_avg = np.where(w.gamma_f, rho_sum + R_m, 0.0) / m
            T_avg = (T_sum + Tf_m) / m
            s = (self.rhoc_fict * w.mass_f * (Tf_m - T_start) / Dt
                 + self.k_fict * (K1 @ T_avg) - rho_avg)
            Tc_new, Rc, itc = implicit_step(c, mat, self.Tc, Dt, Fc_out + w.P.T @ s, None,
                                            self.bottom_c, np.full(c.n_nodes, mat.T_bottom),
                                            T_guess=guess_c, tol=self.newton_tol,
                                            maxit=opts.newton_max,
                                            surface=self.surf_coarse(w.area_out), fict=fict)
            self.stats["newton_coarse"] += itc
            self.stats["coarse_solves"] += 1
            d = np.where(w.gamma_c, Tc_new - lam, 0.0)
            diff = float(np.max(np.abs(d))) if w.gamma_c.any() else 0.0
            theta = self.relaxation(it, d, d_prev, theta)
            d_prev = d
            lam = lam + theta * d
            guess_f, guess_c = Tf_m, Tc_new
            if diff <= self.dn_tol:
                break
        else:
            raise NoConvergence("two-level iteration did not converge")
        self._finish(Tf_m, R_m, Tc_new, Rc, it, Ff, Fc_out, absorbed, bottom, surface,
                     E_start)

    def _step_alternate(self, spots, Fc_all, E_start):
        """A macro step with the alternate global formulation of Section 3:
        the global problem over the whole plate with the global law and only
        the interface jump term, (kappa+ - kappa-) dT-/dn on gamma, which is
        zero here since both levels share kappa(T); the global step is then
        the coarse implicit step itself, and the local problem takes all m
        micro steps with the time-blended Dirichlet data (Algorithm 1, with
        no correction to iterate).  T+ is the global solution everywhere.
        The ledger is the global problem's: stored = sum m_J H+(T+_J),
        absorbed = the global load, bottom = the global bottom reactions,
        surface = the global top-surface loss."""
        opts, mat, c, w = self.opts, self.mat, self.coarse, self.win
        n, m, Dt = self.n, opts.m_time, opts.dt_coarse
        dt = Dt / m
        surf_c = self.surf_coarse(self.area_c)
        Tnew, Rc, it = implicit_step(c, self.mat_global, self.Tc, Dt, Fc_all, None,
                                     self.bottom_c, np.full(c.n_nodes, mat.T_bottom),
                                     tol=self.newton_tol, maxit=opts.newton_max,
                                     surface=surf_c)
        self.stats["newton_coarse"] += it
        self.stats["coarse_solves"] += 1
        PTn, PTp = w.P @ self.Tc, w.P @ Tnew
        T_prev = self.Tf
        for j in range(1, m + 1):
            g = (1.0 - j / m) * PTn + (j / m) * PTp
            T_prev, _ = self.fine_step(T_prev, dt, self.fine_load(spots[j - 1]), g)
        self.Tc = Tnew
        self.Tf = T_prev
        self.n += 1
        absorbed = Dt * Fc_all.sum()
        bottom = -Dt * Rc[self.bottom_c].sum()
        surface = Dt * surf_c.loss(Tnew)
        E_end = self.energy()
        self.ledger["stored"] = E_end
        self.ledger["absorbed"] += absorbed
        self.ledger["bottom"] += bottom
        self.ledger["surface"] += surface
        self.history.append(dict(n=self.n, E_start=E_start, E_end=E_end, absorbed=absorbed,
                                 bottom=bottom, surface=surface, dn_iters=0,
                                 origin=(w.I0, w.J0)))

    def composite_correction(self, T_prev, dt, Ff, rho_sum, Fc_out, guess_f, guess_c):
        """The two-level correction at t_{n+1} as one nonlinear solve on the
        composite grid -- the coarse nodes outside the window's interior
        (interface nodes included) together with the free fine nodes, the
        fine interface values slaved to the coarse ones, T-_gamma = P T+_Gamma.
        Its equations are those that the Dirichlet-Neumann iteration holds at
        its fixed point: R-(T-) = 0 on the free fine rows, and on the free
        coarse rows the outside residual plus the reactions of all m micro
        steps restricted by P^T and averaged, (1/m) sum_j P^T rho_j = 0 --
        so the solution is the same, without the outer iteration.

        With the fine rows scaled by 1/m and z the composite unknowns, the
        residual is G(z) = (1/m) Q^T R-(Q z) + C^T R+(C z) (+ the fixed
        reactions of steps 1..m-1), Q and C the maps from z to the fine and
        coarse fields, and the frozen-kappa Jacobian (1/m) Q^T J- Q + C^T J+ C
        is symmetric positive definite.  Newton with the backtracking of
        oracle.level, stopped when the step taken is within tol.  Returns
        (T-, R-, T+, R+, iterations); T+ holds the injected fine values at the
        window-interior nodes, R- the fine residual with the reactions, R+ the
        coarse outside residual with the restricted reactions (the bottom rows
        of both give the heat leaving through the plate bottom)."""
        w, c, mat, opts = self.win, self.coarse, self.mat, self.opts
        m, Dt = opts.m_time, opts.dt_coarse
        f = w.fine
        free_f = np.flatnonzero(~w.dir_f)
        free_c = np.flatnonzero(~(self.bottom_c | w.interior_c))
        nf, nc = free_f.size, free_c.size
        Pg = w.P[np.flatnonzero(w.gamma_f)]          # fine interface rows
        gam = np.flatnonzero(w.gamma_f)
        # z -> fine field (free rows: identity, interface rows: P), z -> coarse
        Pz = Pg[:, free_c]
        Q = (sp.csr_matrix((np.ones(nf), (free_f, np.arange(nf))), shape=(f.n_nodes, nf + nc))
             + sp.csr_matrix((Pz.data, (gam[np.repeat(np.arange(Pz.shape[0]),
                                                        np.diff(Pz.indptr))],
                                        Pz.indices + nf)), shape=(f.n_nodes, nf + nc)))
        C = sp.csr_matrix((np.ones(nc), (free_c, nf + np.arange(nc))), shape=(c.n_nodes, nf + nc))
        base_c = np.where(self.bottom_c, mat.T_bottom, 0.0)
        # fixed part of the fields: T_bottom on the bottom rows, and its share
        # in the interface values of a window that reaches the bottom
        base_f = np.where(w.bottom_f, mat.T_bottom, 0.0)
        base_f[gam] = Pg @ base_c
        ones_f = np.ones(f.n_elems)
        mass_f, mass_c = w.mass_f, w.mass_out
        sf, sc = self.surf_fine(), self.surf_coarse(w.area_out)
        fixed = (w.P.T @ np.where(w.gamma_f, rho_sum, 0.0)) / m

        def fields(z):
            return base_f + Q @ z, base_c + C @ z

        def evaluate(z):
            Tf, Tc = fields(z)
            Rf, Kf = residual(f, mat, Tf, T_prev, dt, Ff, ones_f, mass_f, sf)
            Rc, Kc = residual(c, mat, Tc, self.Tc, Dt, Fc_out, w.outside_e, mass_c, sc)
            # coarse rows with the restricted reactions of all m micro steps
            Rc = Rc + fixed + (w.P.T @ np.where(w.gamma_f, Rf, 0.0)) / m
            G = (Q.T @ np.where(w.gamma_f, 0.0, Rf)) / m + C.T @ Rc
            return G, Tf, Tc, Rf, Rc, Kf, Kc

        z = np.concatenate([guess_f[free_f], guess_c[free_c]])
        G, Tf, Tc, Rf, Rc, Kf, Kc = evaluate(z)
        for it in range(1, opts.newton_max + 1):
            df = mass_f * M.enthalpy_slope(Tf, mat) / dt
            dc = mass_c * M.enthalpy_slope(Tc, mat) / Dt
            if sf.active:
                df = df + sf.slope(Tf)
            if sc.active:
                dc = dc + sc.slope(Tc)
            A = (Q.T @ (Kf + sp.diags(df)) @ Q) / m + C.T @ (Kc + sp.diags(dc)) @ C
            delta = solve_spd(A.tocsr(), G)
            if not np.all(np.isfinite(delta)):
                raise NoConvergence("non-finite composite Newton update")
            g0 = np.linalg.norm(G)
            dmax = np.max(np.abs(delta)) if delta.size else 0.0
            for h in range(LINE_SEARCH_MAX):
                alpha = 0.5 ** h
                z_try = z - alpha * delta
                trial = evaluate(z_try)
                if np.linalg.norm(trial[0]) <= (1.0 - 1e-4 * alpha) * g0 or alpha * dmax <= self.newton_tol:
                    break
            z = z_try
            G, Tf, Tc, Rf, Rc, Kf, Kc = trial
            if alpha * dmax <= self.newton_tol:
                break
        else:
            raise NoConvergence("composite Newton did not converge")
        self.stats["newton_fine"] += it
        self.stats["fine_solves"] += 1
        Tc = Tc.copy()
        Tc[w.inject_c] = Tf[w.inject_f]
        return Tf, Rf, Tc, Rc, 1

    def _finish(self, Tf_m, R_m, Tc_new, Rc, it, Ff, Fc_out, absorbed, bottom, surface,
                E_start):
        """Ledger terms of the last fine step and the coarse outside step,
        and the commit of the new state."""
        w, opts = self.win, self.opts
        m, Dt = opts.m_time, opts.dt_coarse
        dt = Dt / m
        sf = self.surf_fine()
        self.stats["dn_iters"] += it
        bottom -= dt * R_m[w.bottom_f].sum()
        absorbed += dt * Ff.sum()
        surface += dt * sf.loss(Tf_m)
        bottom -= Dt * Rc[self.bottom_c].sum()
        absorbed += Dt * Fc_out.sum()
        surface += Dt * self.surf_coarse(w.area_out).loss(Tc_new)
        self.Tc = Tc_new
        self.Tf = Tf_m
        if self.record is not None:
            self.record.append((self.n, m, Tf_m.copy()))
        self.n += 1
        E_end = self.energy()
        self.ledger["stored"] = E_end
        self.ledger["absorbed"] += absorbed
        self.ledger["bottom"] += bottom
        self.ledger["surface"] += surface
        self.history.append(dict(n=self.n, E_start=E_start, E_end=E_end, absorbed=absorbed,
                                 bottom=bottom, surface=surface, dn_iters=it,
                                 origin=(w.I0, w.J0)))

    def run(self, n_macro):
        for _ in range(n_macro):
            self.step()
        return self

    def fine_origin(self):
        r = self.mesh.refine
        return (r * self.win.I0, r * self.win.J0, r * self.win.K0)


def run(wl, n_macro=None, **kw):
    sim = TwoLevel(wl, **kw)
    sim.run(wl.n_macro if n_macro is None else n_macro)
    return sim


def single_level_run(grid, mat, scan, dt, n_steps, t_start=None, nq=3, tol=1e-10, T0=None,
                     radiation=False):
    """Plain backward-Euler run of one level over all elements with Dirichlet
    T_bottom at z = z0 and the surface load at each new time level; the top
    surface loses heat by convection (and radiation when `radiation`) as the
    material says.  Returns the list of nodal fields after every step."""
    surf = S.Surface(S.top_area(grid), mat.h_conv, mat.emissivity if radiation else 0.0,
                     mat.T_amb)
    _, _, k = grid.node_ijk()
    bottom = k == 0
    T = np.full(grid.n_nodes, mat.T_init) if T0 is None else np.array(T0, dtype=np.float64)
    T[bottom] = mat.T_bottom
    t0 = scan.t_start if t_start is None else t_start
    out = []
    for s in range(1, n_steps + 1):
        F = L.top_load(grid, L.laser_at(scan, t0 + s * dt), nq)
        T, _, _ = implicit_step(grid, mat, T, dt, F, None, bottom,
                                np.full(grid.n_nodes, mat.T_bottom), tol=tol, surface=surf)
        out.append(T.copy())
    return out
