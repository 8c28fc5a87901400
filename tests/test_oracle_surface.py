"""Pins of the top-surface heat loss (paper Section 2: convection on both
levels' upper surface, radiation on the local one):
  * lumped areas: every top face gives a quarter of its area to each corner;
  * the flux's slope against a central difference;
  * steady state through a slab with constant coefficients: a Dirichlet
    bottom and a convecting and radiating top give a linear profile whose
    top temperature solves one scalar equation -- Q1 reproduces linear
    fields exactly, so the step with a huge time step meets it to roundoff;
  * the energy ledger closes with the surface loss (two levels, window
    moves, convection and radiation);
  * refinement 1, m = 1 with convection still equals the single-level solve
    (the paper's Section 5.1 identity; radiation, local only, is off)."""
from dataclasses import replace

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from oracle import grid as G
from oracle import level as LV
from oracle import surface as S
from oracle import twolevel as TW
from workloads import default_material, small_cases


def test_top_area_lumping():
    g = G.Grid(4, 3, 2, 2e-6, 3e-6, 5e-6)
    A = S.top_area(g)
    i, j, k = g.node_ijk()
    assert A.sum() == pytest.approx(4 * 2e-6 * 3 * 3e-6, rel=1e-14)
    assert np.all(A[k < g.nz] == 0.0)
    face = 2e-6 * 3e-6
    top = k == g.nz
    inner = top & (i > 0) & (i < g.nx) & (j > 0) & (j < g.ny)
    corner = top & ((i == 0) | (i == g.nx)) & ((j == 0) | (j == g.ny))
    assert np.allclose(A[inner], face)
    assert np.allclose(A[corner], face / 4)
    # masking the faces with fi < 2 removes exactly their share
    fj, fi = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
    Am = S.top_area(g, (fi.ravel() >= 2))
    assert Am.sum() == pytest.approx(2 * 3 * face, rel=1e-14)
    assert np.all(Am[top & (i < 2)] == 0.0)


def test_flux_slope_is_derivative():
    T = np.linspace(250.0, 3000.0, 17)
    d = 1e-3
    fd = (S.flux(T + d, 25.0, 0.6, 300.0) - S.flux(T - d, 25.0, 0.6, 300.0)) / (2 * d)
    assert np.allclose(S.flux_slope(T, 25.0, 0.6, 300.0), fd, rtol=1e-8)
    assert S.flux(300.0, 25.0, 0.6, 300.0) == 0.0


@pytest.mark.parametrize("h, eps", [(2.0e4, 0.0), (0.0, 0.9), (5.0e3, 0.7)])
def test_steady_slab_meets_scalar_balance(h, eps):
    """Constant kappa, no latent heat, no laser: the steady field of a slab
    with T_b at the bottom and loss q(T) at the top is linear in z, with
    kappa (T_b - T_top) / L = q(T_top)."""
    kappa, L, Tb, Ta = 15.0, 0.2e-3, 1500.0, 300.0
    mat = default_material(k_lo=kappa, k_hi=kappa, latent=0.0, c_lo=500.0, c_hi=500.0,
                           h_conv=h, emissivity=eps, T_amb=Ta)
    g = G.Grid(3, 2, 8, 20e-6, 25e-6, L / 8)
    _, _, k = g.node_ijk()
    bottom = k == 0
    surf = S.Surface(S.top_area(g), h, eps, Ta)
    T0 = np.full(g.n_nodes, Tb)
    # a step of 1e12 s: the storage term is ~1e-14 of the flux terms
    T, R, _ = LV.implicit_step(g, mat, T0, 1e12, np.zeros(g.n_nodes), None, bottom,
                               np.full(g.n_nodes, Tb), tol=1e-12, surface=surf)
    Ttop = brentq(lambda t: kappa * (Tb - t) / L - S.flux(t, h, eps, Ta), Ta, Tb, xtol=1e-13)
    z = k * (L / 8)
    expect = Tb + (Ttop - Tb) * z / L
    assert np.abs(T - expect).max() < 1e-8 * Tb
    # the bottom reaction carries the whole surface loss out of the slab
    assert -R[bottom].sum() == pytest.approx(-surf.loss(T), rel=1e-9)


def _with_loss(wl, h, eps):
    return replace(wl, material=replace(wl.material, h_conv=h, emissivity=eps, T_amb=300.0))


@pytest.mark.parametrize("name", ["c0", "r3m2"])
def test_energy_ledger_with_surface_loss(name):
    wl = _with_loss(small_cases()[name], 2.0e4, 0.8)
    sim = oracle.run(wl, min(wl.n_macro, 6))
    assert sim.stats["moves"] >= 1 or name == "r3m2"
    for h in sim.history:
        lhs = h["E_end"] - h["E_start"]
        rhs = h["absorbed"] - h["bottom"] - h["surface"]
        assert abs(lhs - rhs) < 1e-9 * h["absorbed"]
        assert h["surface"] > 0.0
    led = sim.ledger
    assert led["stored"] - led["stored0"] == pytest.approx(
        led["absorbed"] - led["bottom"] - led["surface"] + led["remap"], rel=1e-9)


def test_refinement1_identity_with_convection():
    wl = _with_loss(small_cases()["r1m1"], 5.0e4, 0.0)
    n = 6
    sim = TW.TwoLevel(wl)
    ref = TW.single_level_run(sim.coarse, wl.material, wl.scan, wl.options.dt_coarse, n,
                              tol=1e-11)
    for s in range(n):
        sim.step()
        assert np.abs(sim.Tc - ref[s]).max() < 1e-7
    assert sim.stats["moves"] >= 1
    # the loss actually matters at this h
    plain = TW.single_level_run(sim.coarse, replace(wl.material, h_conv=0.0), wl.scan,
                                wl.options.dt_coarse, n, tol=1e-11)
    assert np.abs(plain[-1] - ref[-1]).max() > 1e-3
