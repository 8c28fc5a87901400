"""Pins of one implicit step: manufactured-solution convergence through the
latent band, and the analytic temperature of a Gaussian surface source on a
half-space (constant coefficients, no latent heat)."""
import numpy as np
import pytest

from oracle import grid as G
from oracle import laser as L
from oracle import level as LV
from oracle import material as M
from workloads import Material

UM = 1e-6


# ---------------------------------------------------------------- MMS ------
LX, LY, LZ = 1.0e-3, 0.8e-3, 0.6e-3
T_END = 0.02
MMS_MAT = Material(sharpness=0.01)


def _mms_fields(x, y, z, t):
    """T*(x,t) = 300 + A(t) phi(x), phi = (1 + cos(ax x) cos(ay y))/2 sin(b z),
    A = 1500 t / T_END: insulated sides and top, 300 K at the bottom, sweeping
    300 -> 1800 K through the latent band.  Returns T*, dT*/dt, |grad T*|^2,
    laplacian T*."""
    ax, ay, b = np.pi / LX, np.pi / LY, np.pi / (2 * LZ)
    A, dA = 1500.0 * t / T_END, 1500.0 / T_END
    cx, cy, sz = np.cos(ax * x), np.cos(ay * y), np.sin(b * z)
    g = 0.5 * (1 + cx * cy)
    phi = g * sz
    px = -0.5 * ax * np.sin(ax * x) * cy * sz
    py = -0.5 * ay * cx * np.sin(ay * y) * sz
    pz = g * b * np.cos(b * z)
    lap = -0.5 * (ax ** 2 + ay ** 2) * cx * cy * sz - b * b * g * sz
    return 300.0 + A * phi, dA * phi, A * A * (px * px + py * py + pz * pz), A * lap


def _mms_source(x, y, z, t, mat):
    """Q = dH(T*)/dt - div(kappa(T*) grad T*)."""
    T, Tt, g2, lap = _mms_fields(x, y, z, t)
    dk = np.where((T > mat.T_lo) & (T < mat.T_hi), (mat.k_hi - mat.k_lo) / (mat.T_hi - mat.T_lo), 0.0)
    return M.enthalpy_slope(T, mat) * Tt - dk * g2 - M.conductivity(T, mat) * lap


def _mms_error(n, steps):
    g = G.Grid(n, n, n, LX / n, LY / n, LZ / n)
    x, y, z = g.node_xyz()
    _, _, k = g.node_ijk()
    bottom = k == 0
    m = G.lumped_mass(g)
    T = _mms_fields(x, y, z, 0.0)[0]
    tau = T_END / steps
    for s in range(1, steps + 1):
        t = s * tau
        F = m * _mms_source(x, y, z, t, MMS_MAT)
        T, _, _ = LV.implicit_step(g, MMS_MAT, T, tau, F, None, bottom,
                                   np.full(g.n_nodes, 300.0), tol=1e-9)
    return np.abs(T - _mms_fields(x, y, z, T_END)[0]).max()


def test_mms_second_order():
    errs = [_mms_error(n, s) for n, s in ((4, 2), (8, 8), (16, 32))]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 1.8 <= rates[-1] <= 2.2, (errs, rates)
    assert errs[-1] < errs[0] / 10


# ------------------------------------------------- analytic Gaussian ------
def _half_space_rise(x, y, z_depth, t, P, R, eta, rho_c, kappa):
    """Temperature rise of a stationary Gaussian surface source of absorbed
    power eta P (flux 3 eta P/(pi R^2) exp(-3 r^2/R^2)) switched on at t=0 on
    an insulated half-space: the time integral of the instantaneous point
    response (in-plane variance sigma^2 + 2 alpha s, doubled depth kernel),
    integrated over s = t - t' with the substitution s = u^2."""
    alpha = kappa / rho_c
    sig2 = R * R / 6.0
    u, w = np.polynomial.legendre.leggauss(200)
    umax = np.sqrt(t)
    u = 0.5 * umax * (u + 1)
    w = 0.5 * umax * w
    s = u * u
    r2 = x * x + y * y
    val = (eta * P / (rho_c * np.pi * (sig2 + 2 * alpha * s) * np.sqrt(4 * np.pi * alpha * s))
           * np.exp(-r2 / (2 * (sig2 + 2 * alpha * s)) - z_depth ** 2 / (4 * alpha * s)))
    return float(np.sum(w * 2 * u * val))


def _gauss_error(h, hz, steps):
    mat = Material(c_lo=500.0, c_hi=500.0, k_lo=20.0, k_hi=20.0, latent=0.0)
    P, R, eta, t_end = 4.0, 50 * UM, 1.0, 40 * UM
    lx, lz = 120 * UM, 100 * UM
    g = G.Grid(int(round(lx / h)), int(round(lx / h)), int(round(lz / hz)), h, h, hz)
    _, _, k = g.node_ijk()
    bottom = k == 0
    spot = (0.0, 0.0, P, R, eta, 0)      # beam on the corner: a quarter of it
    T = np.full(g.n_nodes, 300.0)
    tau = t_end / steps
    F = L.top_load(g, spot, 3)
    through_bottom = 0.0
    for _ in range(steps):
        T, Res, _ = LV.implicit_step(g, mat, T, tau, F, None, bottom, np.full(g.n_nodes, 300.0),
                                   tol=1e-10)
        through_bottom += tau * Res[bottom].sum()
    x, y, z = g.node_xyz()
    probes = [(0, 0, g.nz), (2, 1, g.nz), (0, 0, g.nz - 2), (3, 3, g.nz - 1)]
    errs, rises = [], []
    for (i, j, kk) in probes:
        n = g.node(i, j, kk)
        ref = _half_space_rise(x[n], y[n], lz - z[n], t_end, P, R, eta, mat.rho * 500.0, 20.0)
        errs.append(abs(T[n] - 300.0 - ref))
        rises.append(ref)
    # the energy taken in is exactly the absorbed quarter of the beam
    stored = G.lumped_mass(g) @ (M.enthalpy(T, mat) - M.enthalpy(np.full(g.n_nodes, 300.0), mat))
    return (max(errs), max(rises), stored, F.sum() * t_end + through_bottom,
            0.25 * eta * P * t_end)


def test_gaussian_surface_source_half_space():
    e1, rise, st1, ab1, exact = _gauss_error(10 * UM, 5 * UM, 10)
    e2, _, st2, ab2, _ = _gauss_error(5 * UM, 2.5 * UM, 40)
    assert rise > 100.0
    assert e2 < 0.02 * rise
    assert e2 < e1 / 2.5
    # energy balance: stored = absorbed + (tiny) reaction at the cold bottom;
    # the absorbed energy tends to the quarter beam eta P t / 4
    assert st1 == pytest.approx(ab1, rel=1e-9)
    assert st2 == pytest.approx(ab2, rel=1e-9)
    assert ab2 == pytest.approx(exact, rel=1e-5)
