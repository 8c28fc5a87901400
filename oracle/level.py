"""One implicit time step of one level (backward Euler, enthalpy form).

The paper leaves the time integrator open (Section 4: the scheme is not tied
to a particular integrator).  Reading adopted: backward Euler on both levels.
For a level with element set E, lumped mass m^E, Dirichlet nodes D with
values g, and load F evaluated at the new time, the step from T_old with
step tau solves R(T) = 0 on the free nodes, where

    R_i(T) = m_i^E (H(T_i) - H(T_old,i)) / tau
             + sum_{e in E, e contains i} kappa(Tbar_e) (K_e T_e)_i - F_i,

Tbar_e being the mean of the element's 8 nodal temperatures.  The nonlinear
iteration is the "frozen-kappa" Newton method: J = diag(m H'(T) / tau) +
K[kappa(Tbar)], i.e. the exact enthalpy slope on the diagonal with the
kappa' term dropped, which keeps J symmetric positive definite.  The paper
only says the levels are solved to convergence (Section 3); it does not name
the nonlinear scheme.  Plain Newton can cycle when a node crosses the sharp
latent-heat peak of H', so each step T <- T - alpha delta takes the first
alpha in 1, 1/2, 1/4, ... that lowers the 2-norm of the free-row residual by
the factor (1 - 1e-4 alpha) (backtracking line search).  The iteration
stops once the step actually taken satisfies max |alpha delta| <= tol.  The reaction at a Dirichlet node is R_i evaluated at
the converged temperature.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import grid as G
from . import material as M


class NoConvergence(RuntimeError):
    pass


# Halvings tried by the backtracking line search before a step is taken
# regardless (the last, smallest trial is then accepted).
LINE_SEARCH_MAX = 12


class Fictitious:
    """Elements of a level that carry constant coefficients in place of the
    material law -- the global problem's own coefficients inside the local
    domain in the consistent formulation of Section 3: conductivity `kappa`
    [W/m/K] and volumetric heat capacity `rhoc` [J/m3/K] on the elements
    where `elems` is 1.  Their lumped mass enters the time term with rhoc
    (T - T_old) / tau instead of H(T) - H(T_old)."""

    def __init__(self, grid, elems, kappa, rhoc):
        self.elems = np.asarray(elems, dtype=np.float64)
        self.kappa = float(kappa)
        self.rhoc = float(rhoc)
        self.mass = G.lumped_mass(grid, self.elems)


def residual(grid, mat, T, T_old, tau, load, elem_mask, mass, surface=None, fict=None):
    kap = M.conductivity(G.element_mean(grid, T), mat) * elem_mask
    if fict is not None:
        kap = np.where(fict.elems > 0, fict.kappa, kap)
    K = G.stiffness(grid, kap)
    R = mass * (M.enthalpy(T, mat) - M.enthalpy(T_old, mat)) / tau + K @ T - load
    if fict is not None:
        R = R + fict.mass * fict.rhoc * (T - T_old) / tau
    if surface is not None and surface.active:
        R = R + surface.term(T)
    return R, K


def solve_spd(A, b):
    """Solve the SPD system A x = b: direct on small systems, else CG with
    a Jacobi preconditioner to relative residual 1e-13."""
    n = A.shape[0]
    if n == 0:
        return np.zeros(0)
    if n <= 200:
        return spla.spsolve(A.tocsc(), b)
    dinv = 1.0 / A.diagonal()
    Minv = spla.LinearOperator((n, n), matvec=lambda v: dinv * v)
    x, info = spla.cg(A, b, rtol=1e-13, atol=0.0, maxiter=20000, M=Minv)
    if info != 0:
        raise NoConvergence(f"CG did not converge (info={info})")
    return x


def implicit_step(grid, mat, T_old, tau, load, elem_mask=None,
                  dirichlet=None, dirichlet_values=None, T_guess=None,
                  tol=1e-10, maxit=30, surface=None, fict=None):
    """Backward-Euler step of one level.  Returns (T, R, iterations) with R
    the residual at the converged T (reactions on Dirichlet rows, ~0 on free
    rows).  `surface` (oracle.surface.Surface) adds the top-surface heat
    loss A q(T) to the residual and A q'(T) to the Jacobian diagonal.
    `fict` (Fictitious) gives some elements constant coefficients; the
    material law then applies on the other elements of elem_mask only."""
    if elem_mask is None:
        elem_mask = np.ones(grid.n_elems)
    elem_mask = np.asarray(elem_mask, dtype=np.float64)
    if fict is not None:
        elem_mask = elem_mask * (1.0 - fict.elems)
    mass = G.lumped_mass(grid, elem_mask)
    if dirichlet is None:
        dirichlet = np.zeros(grid.n_nodes, dtype=bool)
    T = np.array(T_old if T_guess is None else T_guess, dtype=np.float64)
    if dirichlet_values is not None:
        T[dirichlet] = np.asarray(dirichlet_values)[dirichlet]
    free = np.flatnonzero(~dirichlet)
    R, K = residual(grid, mat, T, T_old, tau, load, elem_mask, mass, surface, fict)
    for it in range(1, maxit + 1):
        diag = mass * M.enthalpy_slope(T, mat) / tau
        if fict is not None:
            diag = diag + fict.mass * fict.rhoc / tau
        if surface is not None and surface.active:
            diag = diag + surface.slope(T)
        J = K + sp.diags(diag)
        Jff = J[free][:, free]
        delta = solve_spd(Jff.tocsr(), R[free])
        if not np.all(np.isfinite(delta)):
            raise NoConvergence("non-finite Newton update")
        # backtracking on the free-row residual norm
        r0 = np.linalg.norm(R[free])
        dmax = np.max(np.abs(delta)) if delta.size else 0.0
        for h in range(LINE_SEARCH_MAX):
            alpha = 0.5 ** h
            T_try = T.copy()
            T_try[free] -= alpha * delta
            R_try, K_try = residual(grid, mat, T_try, T_old, tau, load, elem_mask, mass,
                                    surface, fict)
            if (np.linalg.norm(R_try[free]) <= (1.0 - 1e-4 * alpha) * r0
                    or alpha * dmax <= tol):
                break
        T, R, K = T_try, R_try, K_try
        if alpha * dmax <= tol:
            return T, R, it
    raise NoConvergence(f"Newton did not reach {tol} K in {maxit} iterations")
